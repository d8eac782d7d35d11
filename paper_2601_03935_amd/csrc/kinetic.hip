// Kinetic-step kernels for gfx950: limited gradients, residual with upwind fluxes and the relaxation
// source, Jacobi sweeps of the first-order implicit operator, moments, wall re-emission, boundary flux
// moments, synchronisation and equilibrium initialisation.
//
// Mapping: lanes run over the discrete velocities (or ordinates) of one cell, so every row
// f[cell][slot][0..nv) is read and written with unit stride.  The vector kernels over velocities
// (gradients, residual, sweeps, synchronisation) give each wavefront one chunk of 64 x VW velocities of one
// cell (VW values of 16 bytes per lane) and end it there: many short waves, no loop-carried waits.  The
// moment reduction gives each cell a 4-wave workgroup; the scalar fallbacks and the ordinate kernels use
// one wavefront per cell looping over chunks of 64.  Per-cell geometry and coefficients are wave-uniform
// and live in scalar registers.  Workgroups are remapped so that each of the 8 XCDs walks a contiguous
// range of (Morton-ordered) cells and finds neighbour rows in its own L2.
#include <algorithm>

#include "gsis_dev.h"
#include "gsis_kernels.h"

namespace gsis {

__device__ __forceinline__ int uni_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// magnitudes below this are treated as zero by the limiter (their reciprocal would overflow)
template <typename T>
__device__ __forceinline__ constexpr T tiny_val();
template <>
__device__ __forceinline__ constexpr float tiny_val<float>()
{
    return 1e-30f;
}
template <>
__device__ __forceinline__ constexpr double tiny_val<double>()
{
    return 1e-290;
}

template <typename T>
__device__ __forceinline__ T dexp(T x);
template <>
__device__ __forceinline__ float dexp<float>(float x)
{
    return __expf(x);
}
template <>
__device__ __forceinline__ double dexp<double>(double x)
{
    return exp(x);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// rho (2 pi T)^(-D/2), the normalisation of a D-dimensional Maxwellian, with a division and a square root
template <int D>
__device__ __forceinline__ double gauss_norm(const double rho, const double T)
{
    const double x = 2 * kPi * T;
    if constexpr (D == 1) return rho / sqrt(x);
    else if constexpr (D == 2) return rho / x;
    else return rho / (x * sqrt(x));
}

// sum over aligned groups of G lanes (butterfly within the group)
template <int G>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// lanes per cell of the moment reduction
constexpr int kMomLanes = 16;

// fixed-order sum over the 4 waves of a 256-thread block of per-wave sums (sh: 4 doubles of shared memory
// per value); every thread gets the same result
__device__ __forceinline__ double block4_sum(double v, double *sh)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// Wave w of a (cell, velocity chunk) grid: cells are taken in groups of G consecutive cells and each group
// is traversed chunk-major (chunk 0 of its cells, then chunk 1, ...), so the rows a wave's neighbours
// touch in the same chunk were read shortly before.  G = 1 is cell-major, G >= ncell fully chunk-major.
// Returns false past the end of the grid.
__device__ __forceinline__ bool wave_cell_chunk(const int w, const int ncell, const int nchunk, const int G,
                                                int &c, int &ch)
{
    const int nfull = ncell / G;
    const int wfull = nfull * G * nchunk;
    if (w < wfull) {
        const int cb = w / (G * nchunk);
        const int rem = w - cb * G * nchunk;
        ch = rem / G;
        c = cb * G + (rem - ch * G);
        return true;
    }
    const int tg = ncell - nfull * G;
    if (tg <= 0) return false;
    const int wt = w - wfull;
    ch = wt / tg;
    c = nfull * G + (wt - ch * tg);
    return ch < nchunk;
}

// ------------------------------------------------------------------ limited gradients of f
template <typename T, int D, int NFM>
__global__ __launch_bounds__(256) void k_grad(const T *__restrict__ f, T *__restrict__ gf, const MeshDev m,
                                              const int nd, const int64_t nv, const int second_order,
                                              const int *__restrict__ cell_list, const int64_t ncl,
                                              const int compact)
{
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & 63;
    const int64_t idx = b * 4 + (threadIdx.x >> 6);
    if (idx >= ncl) return;
    const int c = uni_i(cell_list ? cell_list[idx] : (int)idx);
    const int64_t orow = compact ? idx : c;  // row of the output: list position or cell
    const int nfc = uni_i(m.nfc[c]);
    int nb[NFM];
    T lsq[NFM][D], dxc[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = (s < nfc) ? m.nbr[(int64_t)c * NFM + s] : -1;
        const double *g = m.geo + ((int64_t)c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            dxc[s][a] = (s < nfc) ? (T)g[D + a] : T(0);
            lsq[s][a] = (s < nfc) ? (T)g[3 * D + a] : T(0);
        }
    }
    const T eps2 = (T)m.eps2[c];
    for (int64_t k0 = 0; k0 < nv; k0 += kWave) {
        const int64_t k = k0 + lane;
        if (k >= nv) break;
        for (int d = 0; d < nd; ++d) {
            const T fc = f[((int64_t)c * nd + d) * nv + k];
            T g[D];
#pragma unroll
            for (int a = 0; a < D; ++a) g[a] = T(0);
            T dmax = T(0), dmin = T(0), mag = fabs(fc);
#pragma unroll
            for (int s = 0; s < NFM; ++s) {
                if (nb[s] >= 0) {
                    const T fj = f[((int64_t)nb[s] * nd + d) * nv + k], df = fj - fc;
                    mag = fabs(fj) > mag ? fabs(fj) : mag;
#pragma unroll
                    for (int a = 0; a < D; ++a) g[a] += lsq[s][a] * df;
                    dmax = df > dmax ? df : dmax;
                    dmin = df < dmin ? df : dmin;
                }
            }
            T phi = T(0);
            if (second_order) {
                phi = T(1);
                // eps^2 = (K h)^3 M^2 with M the largest |value| of the stencil, applied to the differences divided by M
                // (no underflow of the squares in FP32 where the distribution is tiny)
                const T inv = mag > tiny_val<T>() ? T(1) / mag : T(0);
#pragma unroll
                for (int s = 0; s < NFM; ++s) {
                    if (s < nfc) {
                        T d2 = T(0);
#pragma unroll
                        for (int a = 0; a < D; ++a) d2 += g[a] * dxc[s][a];
                        if (d2 != T(0)) {
                            const T d1 = d2 > T(0) ? dmax : dmin;
                            const T u1 = d1 * inv, u2 = d2 * inv;
                            T p = (u1 * u1 + eps2 + T(2) * u1 * u2) / (u1 * u1 + T(2) * u2 * u2 + u1 * u2 + eps2);
                            p = p > T(1) ? T(1) : p;
                            phi = p < phi ? p : phi;
                        }
                    }
                }
            }
#pragma unroll
            for (int a = 0; a < D; ++a) gf[((orow * nd + d) * D + a) * nv + k] = phi * g[a];
        }
    }
}

// Vector form of k_grad for nv divisible by VW (each lane owns VW consecutive velocities); same
// arithmetic per velocity, neighbour rows loaded with one 16-byte access per lane.
template <typename T, int VW>
using vec_t = T __attribute__((ext_vector_type(VW)));

// VW consecutive values at p (16-byte aligned when VW > 1)
template <typename T, int VW>
__device__ __forceinline__ void load_vw(const T *p, T *v)
{
    if constexpr (VW == 1) {
        v[0] = p[0];
    } else {
        const vec_t<T, VW> x = *(const vec_t<T, VW> *)p;
#pragma unroll
        for (int e = 0; e < VW; ++e) v[e] = x[e];
    }
}
template <typename T, int VW>
__device__ __forceinline__ void store_vw(T *p, const T *v)
{
    if constexpr (VW == 1) {
        p[0] = v[0];
    } else {
        vec_t<T, VW> x;
#pragma unroll
        for (int e = 0; e < VW; ++e) x[e] = v[e];
        *(vec_t<T, VW> *)p = x;
    }
}
// the same for data read or written once by the kernel (streamed past the caches)
template <typename T, int VW>
__device__ __forceinline__ void load_vw_nt(const T *p, T *v)
{
    if constexpr (VW == 1) {
        v[0] = __builtin_nontemporal_load(p);
    } else {
        const vec_t<T, VW> x = __builtin_nontemporal_load((const vec_t<T, VW> *)p);
#pragma unroll
        for (int e = 0; e < VW; ++e) v[e] = x[e];
    }
}
template <typename T, int VW>
__device__ __forceinline__ void store_vw_nt(T *p, const T *v)
{
    if constexpr (VW == 1) {
        __builtin_nontemporal_store(v[0], p);
    } else {
        vec_t<T, VW> x;
#pragma unroll
        for (int e = 0; e < VW; ++e) x[e] = v[e];
        __builtin_nontemporal_store(x, (vec_t<T, VW> *)p);
    }
}

template <typename T, int D, int NFM, int VW>
__global__ __launch_bounds__(256) void k_grad_v(const T *__restrict__ f, T *__restrict__ gf, const MeshDev m,
                                                const int64_t nv, const int nchunk, const int cgroup,
                                                const int second_order,
                                                const int *__restrict__ cell_list, const int64_t ncl,
                                                const int compact)
{
    using V = vec_t<T, VW>;
    constexpr int ND = (D == 3) ? 3 : 4;
    const int w = uni_i((int)(xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6)));
    int idx, ch;
    if (!wave_cell_chunk(w, (int)ncl, nchunk, cgroup, idx, ch)) return;
    const int64_t k = ((int64_t)ch * kWave + (threadIdx.x & 63)) * VW;
    const int c = uni_i(cell_list ? cell_list[idx] : idx);
    const int64_t orow = compact ? idx : c;  // row of the output: list position or cell
    // padded slots: nbr = INT32_MIN, zero geometry (no gradient term, no limiter test)
    int nb[NFM];
    T lsq[NFM][D], dxc[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = m.nbr[(int64_t)c * NFM + s];
        const double *g = m.geo + ((int64_t)c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            dxc[s][a] = (T)g[D + a];
            lsq[s][a] = (T)g[3 * D + a];
        }
    }
    const T eps2 = (T)m.eps2[c];
    if (k < nv) {
        V fcv[ND], fnv[NFM][ND];
#pragma unroll
        for (int d = 0; d < ND; ++d) fcv[d] = *(const V *)(f + ((int64_t)c * ND + d) * nv + k);
#pragma unroll
        for (int s = 0; s < NFM; ++s)
            if (nb[s] >= 0) {
#pragma unroll
                for (int d = 0; d < ND; ++d) fnv[s][d] = *(const V *)(f + ((int64_t)nb[s] * ND + d) * nv + k);
            }
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            V go[D];
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                const T fc = fcv[d][e];
                T g[D];
#pragma unroll
                for (int a = 0; a < D; ++a) g[a] = T(0);
                T dmax = T(0), dmin = T(0), mag = fabs(fc);
#pragma unroll
                for (int s = 0; s < NFM; ++s) {
                    if (nb[s] >= 0) {
                        const T fj = fnv[s][d][e], df = fj - fc;
                        mag = fabs(fj) > mag ? fabs(fj) : mag;
#pragma unroll
                        for (int a = 0; a < D; ++a) g[a] += lsq[s][a] * df;
                        dmax = df > dmax ? df : dmax;
                        dmin = df < dmin ? df : dmin;
                    }
                }
                T phi = T(0);
                if (second_order) {
                    phi = T(1);
                    // eps^2 = (K h)^3 M^2 with M the largest |value| of the stencil, applied to the differences divided by M
                // (no underflow of the squares in FP32 where the distribution is tiny)
                const T inv = mag > tiny_val<T>() ? T(1) / mag : T(0);
#pragma unroll
                    for (int s = 0; s < NFM; ++s) {
                        if (nb[s] != INT32_MIN) {
                            T d2 = T(0);
#pragma unroll
                            for (int a = 0; a < D; ++a) d2 += g[a] * dxc[s][a];
                            if (d2 != T(0)) {
                                const T d1 = d2 > T(0) ? dmax : dmin;
                                const T u1 = d1 * inv, u2 = d2 * inv;
                            T p = (u1 * u1 + eps2 + T(2) * u1 * u2) / (u1 * u1 + T(2) * u2 * u2 + u1 * u2 + eps2);
                                p = p > T(1) ? T(1) : p;
                                phi = p < phi ? p : phi;
                            }
                        }
                    }
                }
#pragma unroll
                for (int a = 0; a < D; ++a) go[a][e] = phi * g[a];
            }
#pragma unroll
            for (int a = 0; a < D; ++a)
                __builtin_nontemporal_store(go[a], (V *)(gf + ((orow * ND + d) * D + a) * nv + k));
        }
    }
}

// per-cell coefficient block (written by k_prologue) -------------------------------------------------
//   [0..D) u, D invtau, D+1 inv_dt, D+2 radc = k_eff (e_vR - e_R)/rho, D+3 B = sigma_R Tv^4/pi,
//   D+4 inv_dtR, D+5 radd = 4 k_eff e_vR / e_v (extra diagonal of f2),
//   then for X in (t, r, v): inv2T, norm, a[D], gR, bR[D], gV, bV[D], hH
__host__ __device__ constexpr int coef_x(int D) { return 5 + 3 * D; }
__host__ __device__ constexpr int coef_size(int D) { return D + 6 + 3 * coef_x(D); }
// per-cell discrete-conservative corrections, for X in (t, r, v): a0, aq, a[D] of G (times e: a0 + aq c^2 /
// (2 T_X) + a . c), then the scalars of R, V, H (slots of kConsX = 8 values)
constexpr int kConsX = 8;

// relaxation source J for the nd slots at velocity xi (Eq. kinetic_equation with Eq. reference_distribution,
// reduced to D velocity dimensions)
template <typename T, int D>
__device__ __forceinline__ void collision(const T *cf, const T *xi, const T *fk, T *J, const int nd, const T wt,
                                          const T wr, const T wv, const T *kc = nullptr)
{
    T cc[D], c2 = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        cc[a] = xi[a] - cf[a];
        c2 += cc[a] * cc[a];
    }
    const T aG = T(0.5) * T(2 + D), aH = T(0.5) * T(D);
    T Ysum[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int X = 0; X < 3; ++X) {
        const T *p = cf + D + 6 + X * coef_x(D);
        const T inv2T = p[0], norm = p[1];
        const T e = norm * dexp<T>(-c2 * inv2T);
        T s = T(0), br = T(0), bv = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            s += p[2 + a] * cc[a];
            br += p[3 + D + a] * cc[a];
            bv += p[4 + 2 * D + a] * cc[a];
        }
        const T q = c2 * inv2T;
        T G = e * (T(1) + s * (q - aG));
        T R = p[2 + D] * G + br * e;
        T V = p[3 + 2 * D] * G + bv * e;
        T H = p[4 + 3 * D] * e * (T(1) + s * (q - aH));
        if (kc) {
            // discrete-conservative corrections (a multiple of e = rho f0^eq(T_X) per slot)
            const T *k = kc + X * kConsX;
            T P = k[0] + k[1] * q;
#pragma unroll
            for (int a = 0; a < D; ++a) P += k[2 + a] * cc[a];
            G += P * e;
            R += k[D + 2] * e;
            V += k[D + 3] * e;
            H += k[D + 4] * e;
        }
        const T wX = (X == 0) ? wt : ((X == 1) ? wr : wv);
        Ysum[0] += wX * G;
        Ysum[1] += wX * R;
        Ysum[2] += wX * V;
        Ysum[3] += wX * H;
    }
    const T invtau = cf[D];
    for (int d = 0; d < nd; ++d) J[d] = (Ysum[d] - fk[d]) * invtau;
    J[2] -= fk[0] * cf[D + 2];
}

// boundary state on an incoming velocity: equilibrium (rho, u, T) of the tag, rho replaced by the wall
// re-emission density on walls
template <typename T, int D>
__device__ __forceinline__ void boundary_values(const BcDev &bc, const T rho, const T *xi, const T dr, T *out)
{
    T c2 = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const T cc = xi[a] - (T)bc.u[a];
        c2 += cc * cc;
    }
    const T Tb = (T)bc.T;
    const T two_pi_T = T(2.0 * kPi) * Tb;
    T norm = T(1);
#pragma unroll
    for (int a = 0; a < D; ++a) norm *= two_pi_T;
    const T G = rho * dexp<T>(-c2 / (T(2) * Tb)) / sqrt(norm);
    out[0] = G;
    out[1] = T(0.5) * dr * Tb * G;
    out[2] = (T)bc.ev * G;
    out[3] = T(3 - D) * Tb * G;
}

// ------------------------------------------------------------------ residual and first increment
template <typename T, int D, int NFM>
__global__ __launch_bounds__(256) void k_residual(const T *__restrict__ f, const T *__restrict__ gf,
                                                  const T *__restrict__ coef, const T *__restrict__ ccons,
                                                  const T *__restrict__ xi,
                                                  const T *__restrict__ rhow, T *__restrict__ r,
                                                  T *__restrict__ dl, T *__restrict__ fout, const MeshDev m,
                                                  const int64_t nv, const T cflv_fac, const T omega,
                                                  const T wt, const T wr, const T wv, const T dr, const T dv)
{
    constexpr int ND = (D == 3) ? 3 : 4;
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & 63;
    const int64_t ci = b * 4 + (threadIdx.x >> 6);
    if (ci >= m.nc) return;
    const int c = uni_i((int)ci);
    const int nfc = uni_i(m.nfc[c]);
    int nb[NFM];
    T nsv[NFM][D], dxc[NFM][D], dxj[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = (s < nfc) ? m.nbr[(int64_t)c * NFM + s] : INT32_MIN;
        const double *g = m.geo + ((int64_t)c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            nsv[s][a] = (s < nfc) ? (T)g[a] : T(0);
            dxc[s][a] = (s < nfc) ? (T)g[D + a] : T(0);
            dxj[s][a] = (s < nfc) ? (T)g[2 * D + a] : T(0);
        }
    }
    T cf[coef_size(3)];
#pragma unroll
    for (int i = 0; i < coef_size(D); ++i) cf[i] = coef[(int64_t)c * coef_size(D) + i];
    for (int64_t k0 = 0; k0 < nv; k0 += kWave) {
        const int64_t k = k0 + lane;
        if (k >= nv) break;
        T x[D];
#pragma unroll
        for (int a = 0; a < D; ++a) x[a] = xi[k * D + a];
        T fc[ND], gc[ND][D];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            fc[d] = f[((int64_t)c * ND + d) * nv + k];
#pragma unroll
            for (int a = 0; a < D; ++a) gc[d][a] = gf[(((int64_t)c * ND + d) * D + a) * nv + k];
        }
        T flux[ND];
#pragma unroll
        for (int d = 0; d < ND; ++d) flux[d] = T(0);
        T dsum = T(0);
#pragma unroll
        for (int s = 0; s < NFM; ++s) {
            if (nb[s] == INT32_MIN) continue;
            T xn = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) xn += x[a] * nsv[s][a];
            T fv[4];
            if (xn > T(0)) {
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    T v = fc[d];
#pragma unroll
                    for (int a = 0; a < D; ++a) v += gc[d][a] * dxc[s][a];
                    fv[d] = v;
                }
                dsum += xn;
            } else if (nb[s] >= 0) {
                const int64_t j = nb[s];
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    T v = f[(j * ND + d) * nv + k];
#pragma unroll
                    for (int a = 0; a < D; ++a) v += gf[((j * ND + d) * D + a) * nv + k] * dxj[s][a];
                    fv[d] = v;
                }
            } else {
                const int bfi = -nb[s] - 1;
                const BcDev bc = m.bcs[m.bf_tag[bfi]];
                const T rho = (bc.kind == 0) ? rhow[bfi] : (T)bc.rho;
                boundary_values<T, D>(bc, rho, x, dr, fv);
            }
#pragma unroll
            for (int d = 0; d < ND; ++d) flux[d] += xn * fv[d];
        }
        T J[4];
        collision<T, D>(cf, x, fc, J, ND, wt, wr, wv, ccons ? ccons + (int64_t)c * 3 * kConsX : nullptr);
        const T dcoef = cf[D + 1] + cf[D] + dsum * cflv_fac;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const int64_t o = ((int64_t)c * ND + d) * nv + k;
            const T rr = J[d] - flux[d];
            const T dd = (d == 2) ? dcoef + cf[D + 5] : dcoef;
            if (fout) {
                fout[o] = fc[d] + omega * (rr / dd);
            } else {
                r[o] = rr;
                if (dl) dl[o] = rr / dd;
            }
        }
    }
}

// Vector form of k_residual for nv divisible by VW (each lane owns VW consecutive velocities); the
// rows of interior neighbours are loaded for every lane and the upwind choice is made per velocity.
template <typename T, int D, int NFM, int VW>
__global__ __launch_bounds__(256) void k_residual_v(const T *__restrict__ f, const T *__restrict__ gf,
                                                    const T *__restrict__ coef, const T *__restrict__ ccons,
                                                    const T *__restrict__ xiT,
                                                    const T *__restrict__ rhow, T *__restrict__ r,
                                                    T *__restrict__ dl, T *__restrict__ fout, const MeshDev m,
                                                    const int64_t nv, const int nchunk, const int cgroup,
                                                    const T cflv_fac,
                                                    const T omega, const T wt, const T wr, const T wv, const T dr,
                                                    const T dv)
{
    using V = vec_t<T, VW>;
    constexpr int ND = (D == 3) ? 3 : 4;
    const int w = uni_i((int)(xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6)));
    int c, ch;
    if (!wave_cell_chunk(w, (int)m.nc, nchunk, cgroup, c, ch)) return;
    const int64_t k = ((int64_t)ch * kWave + (threadIdx.x & 63)) * VW;
    // padded slots: nbr = INT32_MIN, zero geometry
    int nb[NFM];
    T nsv[NFM][D], dxc[NFM][D], dxj[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = m.nbr[(int64_t)c * NFM + s];
        const double *g = m.geo + ((int64_t)c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            nsv[s][a] = (T)g[a];
            dxc[s][a] = (T)g[D + a];
            dxj[s][a] = (T)g[2 * D + a];
        }
    }
    T cf[coef_size(3)];
#pragma unroll
    for (int i = 0; i < coef_size(D); ++i) cf[i] = coef[(int64_t)c * coef_size(D) + i];
    if (k < nv) {
        V x[D], fc[ND], gc[ND][D];
#pragma unroll
        for (int a = 0; a < D; ++a) x[a] = *(const V *)(xiT + a * nv + k);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            fc[d] = *(const V *)(f + ((int64_t)c * ND + d) * nv + k);
#pragma unroll
            for (int a = 0; a < D; ++a) gc[d][a] = *(const V *)(gf + (((int64_t)c * ND + d) * D + a) * nv + k);
        }
        V flux[ND], dsum = T(0);
#pragma unroll
        for (int d = 0; d < ND; ++d) flux[d] = T(0);
#pragma unroll
        for (int s = 0; s < NFM; ++s) {
            if (nb[s] == INT32_MIN) continue;
            V xn = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) xn += x[a] * nsv[s][a];
            if (nb[s] >= 0) {
                const int64_t j = nb[s];
                // the neighbour's reconstruction enters only where it is upwind (xi . n <= 0): a lane whose
                // velocities all leave through this face does not load the neighbour's rows
                bool up = false;
#pragma unroll
                for (int e = 0; e < VW; ++e) up = up || !(xn[e] > T(0));
                V fj[ND], gj[ND][D];
                if (up) {
#pragma unroll
                    for (int d = 0; d < ND; ++d) {
                        fj[d] = *(const V *)(f + (j * ND + d) * nv + k);
#pragma unroll
                        for (int a = 0; a < D; ++a) gj[d][a] = *(const V *)(gf + ((j * ND + d) * D + a) * nv + k);
                    }
                } else {
#pragma unroll
                    for (int d = 0; d < ND; ++d) {
                        fj[d] = T(0);
#pragma unroll
                        for (int a = 0; a < D; ++a) gj[d][a] = T(0);
                    }
                }
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    T fv[4];
                    if (xn[e] > T(0)) {
#pragma unroll
                        for (int d = 0; d < ND; ++d) {
                            T v = fc[d][e];
#pragma unroll
                            for (int a = 0; a < D; ++a) v += gc[d][a][e] * dxc[s][a];
                            fv[d] = v;
                        }
                        dsum[e] += xn[e];
                    } else {
#pragma unroll
                        for (int d = 0; d < ND; ++d) {
                            T v = fj[d][e];
#pragma unroll
                            for (int a = 0; a < D; ++a) v += gj[d][a][e] * dxj[s][a];
                            fv[d] = v;
                        }
                    }
#pragma unroll
                    for (int d = 0; d < ND; ++d) flux[d][e] += xn[e] * fv[d];
                }
            } else {
                const int bfi = -nb[s] - 1;
                const BcDev bc = m.bcs[m.bf_tag[bfi]];
                const T rho = (bc.kind == 0) ? rhow[bfi] : (T)bc.rho;
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    T fv[4];
                    if (xn[e] > T(0)) {
#pragma unroll
                        for (int d = 0; d < ND; ++d) {
                            T v = fc[d][e];
#pragma unroll
                            for (int a = 0; a < D; ++a) v += gc[d][a][e] * dxc[s][a];
                            fv[d] = v;
                        }
                        dsum[e] += xn[e];
                    } else {
                        T xe[D];
#pragma unroll
                        for (int a = 0; a < D; ++a) xe[a] = x[a][e];
                        boundary_values<T, D>(bc, rho, xe, dr, fv);
                    }
#pragma unroll
                    for (int d = 0; d < ND; ++d) flux[d][e] += xn[e] * fv[d];
                }
            }
        }
        V rr[ND], dd[ND];
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            T xe[D], fe[4], J[4];
#pragma unroll
            for (int a = 0; a < D; ++a) xe[a] = x[a][e];
#pragma unroll
            for (int d = 0; d < ND; ++d) fe[d] = fc[d][e];
            collision<T, D>(cf, xe, fe, J, ND, wt, wr, wv, ccons ? ccons + (int64_t)c * 3 * kConsX : nullptr);
            const T dcoef = cf[D + 1] + cf[D] + dsum[e] * cflv_fac;
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                rr[d][e] = J[d] - flux[d][e];
                dd[d][e] = (d == 2) ? dcoef + cf[D + 5] : dcoef;
            }
        }
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const int64_t o = ((int64_t)c * ND + d) * nv + k;
            if (fout) {
                __builtin_nontemporal_store(fc[d] + omega * (rr[d] / dd[d]), (V *)(fout + o));
            } else {
                __builtin_nontemporal_store(rr[d], (V *)(r + o));
                if (dl) __builtin_nontemporal_store(rr[d] / dd[d], (V *)(dl + o));
            }
        }
    }
}

// ------------------------------------------------------------------ residual with gradients recomputed
// Limited gradient of distribution d of cell j at the lane's VW velocities: the arithmetic of k_grad_v for
// one distribution.  nbj: the NFM neighbour slots of j (>= 0 neighbour, < 0 boundary face, INT32_MIN none);
// fj: f of (j, d) at the lane's velocities.
template <typename T, int D, int NFM, int VW>
__device__ __forceinline__ void limited_grad_v(const T *__restrict__ f, const MeshDev &m, const int j,
                                               const int (&nbj)[NFM], const vec_t<T, VW> fj, const int d,
                                               const int64_t k, const int64_t nv, const int second_order,
                                               vec_t<T, VW> (&go)[D])
{
    using V = vec_t<T, VW>;
    constexpr int ND = (D == 3) ? 3 : 4;
    T lsq[NFM][D], dxc[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        const double *g = m.geo + ((int64_t)j * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            dxc[s][a] = (T)g[D + a];
            lsq[s][a] = (T)g[3 * D + a];
        }
    }
    const T eps2 = (T)m.eps2[j];
    V fn[NFM];
#pragma unroll
    for (int s = 0; s < NFM; ++s)
        if (nbj[s] >= 0) fn[s] = *(const V *)(f + ((int64_t)nbj[s] * ND + d) * nv + k);
#pragma unroll
    for (int e = 0; e < VW; ++e) {
        const T fc = fj[e];
        T g[D];
#pragma unroll
        for (int a = 0; a < D; ++a) g[a] = T(0);
        T dmax = T(0), dmin = T(0), mag = fabs(fc);
#pragma unroll
        for (int s = 0; s < NFM; ++s) {
            if (nbj[s] >= 0) {
                const T fv = fn[s][e], df = fv - fc;
                mag = fabs(fv) > mag ? fabs(fv) : mag;
#pragma unroll
                for (int a = 0; a < D; ++a) g[a] += lsq[s][a] * df;
                dmax = df > dmax ? df : dmax;
                dmin = df < dmin ? df : dmin;
            }
        }
        T phi = T(0);
        if (second_order) {
            phi = T(1);
            const T inv = mag > tiny_val<T>() ? T(1) / mag : T(0);
#pragma unroll
            for (int s = 0; s < NFM; ++s) {
                if (nbj[s] != INT32_MIN) {
                    T d2 = T(0);
#pragma unroll
                    for (int a = 0; a < D; ++a) d2 += g[a] * dxc[s][a];
                    if (d2 != T(0)) {
                        const T d1 = d2 > T(0) ? dmax : dmin;
                        const T u1 = d1 * inv, u2 = d2 * inv;
                        T p = (u1 * u1 + eps2 + T(2) * u1 * u2) / (u1 * u1 + T(2) * u2 * u2 + u1 * u2 + eps2);
                        p = p > T(1) ? T(1) : p;
                        phi = p < phi ? p : phi;
                    }
                }
            }
        }
#pragma unroll
        for (int a = 0; a < D; ++a) go[a][e] = phi * g[a];
    }
}

// The residual of k_residual_v without a stored gradient field: each wave recomputes the limited gradients
// of its cell and of the face neighbours it needs (their neighbour rows, the second ring, come through the
// caches), distribution by distribution, so the kinetic step reads f and writes r (and the first Jacobi
// iterate) with no gradient traffic.  Same arithmetic per velocity as k_grad_v followed by k_residual_v.
template <typename T, int D, int NFM, int VW>
__global__ __launch_bounds__(256) void k_gres_v(const T *__restrict__ f, const T *__restrict__ coef,
                                                const T *__restrict__ ccons, const T *__restrict__ xiT,
                                                const T *__restrict__ rhow,
                                                T *__restrict__ r, T *__restrict__ dl, T *__restrict__ fout,
                                                const MeshDev m, const int64_t nv, const int nchunk,
                                                const int cgroup, const int second_order, const T cflv_fac,
                                                const T omega, const T wt, const T wr, const T wv, const T dr,
                                                const T dv)
{
    using V = vec_t<T, VW>;
    constexpr int ND = (D == 3) ? 3 : 4;
    const int w = uni_i((int)(xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6)));
    int c, ch;
    if (!wave_cell_chunk(w, (int)m.nc, nchunk, cgroup, c, ch)) return;
    const int64_t k = ((int64_t)ch * kWave + (threadIdx.x & 63)) * VW;
    if (k >= nv) return;
    int nb[NFM];
    T nsv[NFM][D], dxc[NFM][D], dxj[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = m.nbr[(int64_t)c * NFM + s];
        const double *g = m.geo + ((int64_t)c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            nsv[s][a] = (T)g[a];
            dxc[s][a] = (T)g[D + a];
            dxj[s][a] = (T)g[2 * D + a];
        }
    }
    T cf[coef_size(3)];
#pragma unroll
    for (int i = 0; i < coef_size(D); ++i) cf[i] = coef[(int64_t)c * coef_size(D) + i];
    V x[D], fc[ND];
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = *(const V *)(xiT + a * nv + k);
#pragma unroll
    for (int d = 0; d < ND; ++d) fc[d] = *(const V *)(f + ((int64_t)c * ND + d) * nv + k);
    // upwind diagonal sum and relaxation source
    V dsum = T(0);
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        if (nb[s] == INT32_MIN) continue;
        V xn = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) xn += x[a] * nsv[s][a];
#pragma unroll
        for (int e = 0; e < VW; ++e)
            if (xn[e] > T(0)) dsum[e] += xn[e];
    }
    V Jv[ND];
#pragma unroll
    for (int e = 0; e < VW; ++e) {
        T xe[D], fe[4], J[4];
#pragma unroll
        for (int a = 0; a < D; ++a) xe[a] = x[a][e];
#pragma unroll
        for (int d = 0; d < ND; ++d) fe[d] = fc[d][e];
        collision<T, D>(cf, xe, fe, J, ND, wt, wr, wv, ccons ? ccons + (int64_t)c * 3 * kConsX : nullptr);
#pragma unroll
        for (int d = 0; d < ND; ++d) Jv[d][e] = J[d];
    }
    for (int d = 0; d < ND; ++d) {
        V gc[D];
        limited_grad_v<T, D, NFM, VW>(f, m, c, nb, fc[d], d, k, nv, second_order, gc);
        V flux = T(0);
#pragma unroll
        for (int s = 0; s < NFM; ++s) {
            if (nb[s] == INT32_MIN) continue;
            V xn = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) xn += x[a] * nsv[s][a];
            if (nb[s] >= 0) {
                const int j = nb[s];
                int nbj[NFM];
#pragma unroll
                for (int t = 0; t < NFM; ++t) nbj[t] = m.nbr[(int64_t)j * NFM + t];
                const V fj = *(const V *)(f + ((int64_t)j * ND + d) * nv + k);
                V gj[D];
                limited_grad_v<T, D, NFM, VW>(f, m, j, nbj, fj, d, k, nv, second_order, gj);
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    T v;
                    if (xn[e] > T(0)) {
                        v = fc[d][e];
#pragma unroll
                        for (int a = 0; a < D; ++a) v += gc[a][e] * dxc[s][a];
                    } else {
                        v = fj[e];
#pragma unroll
                        for (int a = 0; a < D; ++a) v += gj[a][e] * dxj[s][a];
                    }
                    flux[e] += xn[e] * v;
                }
            } else {
                const int bfi = -nb[s] - 1;
                const BcDev bc = m.bcs[m.bf_tag[bfi]];
                const T rho = (bc.kind == 0) ? rhow[bfi] : (T)bc.rho;
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    T v;
                    if (xn[e] > T(0)) {
                        v = fc[d][e];
#pragma unroll
                        for (int a = 0; a < D; ++a) v += gc[a][e] * dxc[s][a];
                    } else {
                        T xe[D], fv[4];
#pragma unroll
                        for (int a = 0; a < D; ++a) xe[a] = x[a][e];
                        boundary_values<T, D>(bc, rho, xe, dr, fv);
                        v = fv[d];
                    }
                    flux[e] += xn[e] * v;
                }
            }
        }
        V rr, dd;
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const T dcoef = cf[D + 1] + cf[D] + dsum[e] * cflv_fac;
            rr[e] = Jv[d][e] - flux[e];
            dd[e] = (d == 2) ? dcoef + cf[D + 5] : dcoef;
        }
        const int64_t o = ((int64_t)c * ND + d) * nv + k;
        if (fout) {
            __builtin_nontemporal_store(fc[d] + omega * (rr / dd), (V *)(fout + o));
        } else {
            __builtin_nontemporal_store(rr, (V *)(r + o));
            if (dl) __builtin_nontemporal_store(rr / dd, (V *)(dl + o));
        }
    }
}

// ------------------------------------------------------------------ Jacobi sweep of the implicit operator
template <typename T, int D, int NFM>
__global__ __launch_bounds__(256) void k_sweep(const T *__restrict__ r, const T *__restrict__ dlin,
                                               T *__restrict__ dlout, const T *__restrict__ f,
                                               T *__restrict__ fout, const T *__restrict__ coef,
                                               const T *__restrict__ xi, const MeshDev m, const int64_t nv,
                                               const T cflv_fac, const T omega)
{
    constexpr int ND = (D == 3) ? 3 : 4;
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & 63;
    const int64_t ci = b * 4 + (threadIdx.x >> 6);
    if (ci >= m.nc) return;
    const int c = uni_i((int)ci);
    const int nfc = uni_i(m.nfc[c]);
    int nb[NFM];
    T nsv[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = (s < nfc) ? m.nbr[(int64_t)c * NFM + s] : INT32_MIN;
        const double *g = m.geo + ((int64_t)c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) nsv[s][a] = (s < nfc) ? (T)g[a] : T(0);
    }
    const T base = coef[(int64_t)c * coef_size(D) + D + 1] + coef[(int64_t)c * coef_size(D) + D];
    const T radd = coef[(int64_t)c * coef_size(D) + D + 5];
    for (int64_t k0 = 0; k0 < nv; k0 += kWave) {
        const int64_t k = k0 + lane;
        if (k >= nv) break;
        T x[D];
#pragma unroll
        for (int a = 0; a < D; ++a) x[a] = xi[k * D + a];
        T acc[ND];
#pragma unroll
        for (int d = 0; d < ND; ++d) acc[d] = T(0);
        T dsum = T(0);
#pragma unroll
        for (int s = 0; s < NFM; ++s) {
            if (nb[s] == INT32_MIN) continue;
            T xn = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) xn += x[a] * nsv[s][a];
            if (xn > T(0)) {
                dsum += xn;
            } else if (xn < T(0) && nb[s] >= 0) {
                const int64_t j = nb[s];
#pragma unroll
                for (int d = 0; d < ND; ++d) acc[d] += xn * dlin[(j * ND + d) * nv + k];
            }
        }
        const T dcoef = base + dsum * cflv_fac;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const int64_t o = ((int64_t)c * ND + d) * nv + k;
            const T dn = (r[o] - acc[d]) / ((d == 2) ? dcoef + radd : dcoef);
            if (fout)
                fout[o] = f[o] + omega * dn;
            else
                dlout[o] = dn;
        }
    }
}

// Vector form of k_sweep for nv divisible by VW.  One wave per (cell, chunk of 64 VW velocities): each
// lane owns VW consecutive velocities (one 16-byte load or store per row and lane) and the wave ends after
// its chunk, so many short waves keep the memory system busy without loop-carried waits.  The rows of all
// upwind neighbours are loaded for every lane and the upwind choice is a per-velocity select.  Same
// arithmetic as k_sweep except the division, done as a multiplication by the reciprocal of the diagonal.
// Padded cell slots hold nbr = INT32_MIN and zero geometry, so the per-cell tables are read without
// waiting for the face count.
template <typename T, int D, int NFM, int VW>
__global__ __launch_bounds__(256) void k_sweep_v(const T *__restrict__ r, const T *__restrict__ dlin,
                                                 T *__restrict__ dlout, const T *__restrict__ f,
                                                 T *__restrict__ fout, const T *__restrict__ coef,
                                                 const T *__restrict__ xiT, const MeshDev m, const int64_t nv,
                                                 const int nchunk, const int cgroup, const T cflv_fac,
                                                 const T omega)
{
    using V = vec_t<T, VW>;
    constexpr int ND = (D == 3) ? 3 : 4;
    const int w = uni_i((int)(xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6)));
    int c, ch;
    if (!wave_cell_chunk(w, (int)m.nc, nchunk, cgroup, c, ch)) return;
    const int64_t k = ((int64_t)ch * kWave + (threadIdx.x & 63)) * VW;
    int nb[NFM];
    T nsv[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = m.nbr[(int64_t)c * NFM + s];
        const double *g = m.geo + ((int64_t)c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) nsv[s][a] = (T)g[a];
    }
    const T base = coef[(int64_t)c * coef_size(D) + D + 1] + coef[(int64_t)c * coef_size(D) + D];
    const T radd = coef[(int64_t)c * coef_size(D) + D + 5];
    if (k >= nv) return;
    V x[D];
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = *(const V *)(xiT + a * nv + k);
    V nbv[NFM][ND];
#pragma unroll
    for (int s = 0; s < NFM; ++s)
        if (nb[s] >= 0) {
#pragma unroll
            for (int d = 0; d < ND; ++d) nbv[s][d] = *(const V *)(dlin + ((int64_t)nb[s] * ND + d) * nv + k);
        }
    V rv[ND];
#pragma unroll
    // r and f are read once per sweep: streamed past the caches, which keep the neighbours' increment rows
    for (int d = 0; d < ND; ++d) rv[d] = __builtin_nontemporal_load((const V *)(r + ((int64_t)c * ND + d) * nv + k));
    V acc[ND], dsum = T(0);
#pragma unroll
    for (int d = 0; d < ND; ++d) acc[d] = T(0);
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        if (nb[s] == INT32_MIN) continue;
        V xn = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) xn += x[a] * nsv[s][a];
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            if (xn[e] > T(0)) {
                dsum[e] += xn[e];
            } else if (xn[e] < T(0) && nb[s] >= 0) {
#pragma unroll
                for (int d = 0; d < ND; ++d) acc[d][e] += xn[e] * nbv[s][d][e];
            }
        }
    }
    V inv0, inv2;
#pragma unroll
    for (int e = 0; e < VW; ++e) {
        const T dc = base + dsum[e] * cflv_fac;
        inv0[e] = T(1) / dc;
        inv2[e] = T(1) / (dc + radd);
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const int64_t o = ((int64_t)c * ND + d) * nv + k;
        const V dn = (rv[d] - acc[d]) * ((d == 2) ? inv2 : inv0);
        if (fout) {
            const V fo = __builtin_nontemporal_load((const V *)(f + o)) + omega * dn;
            __builtin_nontemporal_store(fo, (V *)(fout + o));
        } else {
            __builtin_nontemporal_store(dn, (V *)(dlout + o));
        }
    }
}

// vector load / store of VW consecutive values (16-byte aligned when VW > 1; any alignment for VW = 1)
template <typename T, int VW>
__device__ __forceinline__ vec_t<T, VW> ldv(const T *p)
{
    if constexpr (VW == 1) {
        vec_t<T, 1> v;
        v[0] = p[0];
        return v;
    } else {
        return *(const vec_t<T, VW> *)p;
    }
}
template <typename T, int VW>
__device__ __forceinline__ void stv(T *p, const vec_t<T, VW> v)
{
    if constexpr (VW == 1)
        p[0] = v[0];
    else
        *(vec_t<T, VW> *)p = v;
}

// ------------------------------------------------------------------ colored symmetric Gauss-Seidel passes
// The paper's forward and backward point relaxation of the first-order implicit operator (Sec. 6), taken
// colour by colour: cells of one colour share no face, so one launch updates a whole colour.  With
// a_j = xi_n^- S / V on the face to neighbour j (xi_n < 0) and d the diagonal of the Jacobi kernels:
//   MODE 0, first forward pass:   D_c = (r_c - sum_{j lower} a_j D_j) / d
//   MODE 1, first backward pass:  D_c = D_c - (1 / d) sum_{j upper} a_j D_j
//   MODE 2, later passes:         D_c = (r_c - sum_{all j} a_j D_j) / d
// (lower / upper: the neighbour's colour is below / above the colour q of the launch).  The first symmetric
// sweep starts from D = 0, so MODE 0 + MODE 1 is (D + L) D^-1 (D + U) D = r and needs no separate r: with
// one sweep r and dl are the same buffer (hence no __restrict__ on them).  With update_f, f_c += omega D_c.
// One wave per (cell of the colour list, chunk of 64 VW velocities), as the Jacobi kernel.
template <typename T, int D, int NFM, int VW, int MODE>
__global__ __launch_bounds__(256) void k_sgs_v(const T *r, T *dl, T *__restrict__ f, const T *__restrict__ coef,
                                               const T *__restrict__ xiT, const MeshDev m, const int64_t nv,
                                               const int nchunk, const int cgroup, const T cflv_fac, const T omega,
                                               const int *__restrict__ cells, const int ncl, const int q,
                                               const int update_f)
{
    using V = vec_t<T, VW>;
    constexpr int ND = (D == 3) ? 3 : 4;
    const int w = uni_i((int)(xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6)));
    int idx, ch;
    if (!wave_cell_chunk(w, ncl, nchunk, cgroup, idx, ch)) return;
    const int64_t k = ((int64_t)ch * kWave + (threadIdx.x & 63)) * VW;
    const int c = uni_i(cells[idx]);
    int nb[NFM];
    bool use[NFM];
    T nsv[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = m.nbr[(int64_t)c * NFM + s];
        const double *g = m.geo + ((int64_t)c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) nsv[s][a] = (T)g[a];
        bool u = nb[s] >= 0;
        if (u && MODE != 2) {
            const int qj = m.color[nb[s]];
            u = (MODE == 0) ? (qj < q) : (qj > q);
        }
        use[s] = u;
    }
    const T base = coef[(int64_t)c * coef_size(D) + D + 1] + coef[(int64_t)c * coef_size(D) + D];
    const T radd = coef[(int64_t)c * coef_size(D) + D + 5];
    if (k >= nv) return;
    V x[D];
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = ldv<T, VW>(xiT + a * nv + k);
    V nbv[NFM][ND];
#pragma unroll
    for (int s = 0; s < NFM; ++s)
        if (use[s]) {
#pragma unroll
            for (int d = 0; d < ND; ++d) nbv[s][d] = ldv<T, VW>(dl + ((int64_t)nb[s] * ND + d) * nv + k);
        }
    V own[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d)
        own[d] = ldv<T, VW>((MODE == 1 ? (const T *)dl : r) + ((int64_t)c * ND + d) * nv + k);
    V acc[ND], dsum = T(0);
#pragma unroll
    for (int d = 0; d < ND; ++d) acc[d] = T(0);
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        if (nb[s] == INT32_MIN) continue;
        V xn = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) xn += x[a] * nsv[s][a];
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            if (xn[e] > T(0)) {
                dsum[e] += xn[e];
            } else if (xn[e] < T(0) && use[s]) {
#pragma unroll
                for (int d = 0; d < ND; ++d) acc[d][e] += xn[e] * nbv[s][d][e];
            }
        }
    }
    V inv0, inv2;
#pragma unroll
    for (int e = 0; e < VW; ++e) {
        const T dc = base + dsum[e] * cflv_fac;
        inv0[e] = T(1) / dc;
        inv2[e] = T(1) / (dc + radd);
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const int64_t o = ((int64_t)c * ND + d) * nv + k;
        const V iv = (d == 2) ? inv2 : inv0;
        const V dn = (MODE == 1) ? own[d] - acc[d] * iv : (own[d] - acc[d]) * iv;
        stv<T, VW>(dl + o, dn);
        if (update_f) {
            V fo;
            fo = ldv<T, VW>(f + o);
            fo = fo + omega * dn;
            stv<T, VW>(f + o, fo);
        }
    }
}

// Ordinate form of the colored symmetric Gauss-Seidel pass (same modes), packed like the other ordinate
// kernels: 2^lsh lanes per cell of the colour list, each lane VW consecutive ordinates per step.
template <typename T, int D, int NFM, int VW, int MODE>
__global__ __launch_bounds__(256) void k_sgs_Iv(const T *r, T *dl, T *__restrict__ I, const T *__restrict__ coef,
                                                const T *__restrict__ om, const MeshDev m, const int64_t no,
                                                const int lsh, const T cflv_fac, const T omega, const T keff,
                                                const int *__restrict__ cells, const int ncl, const int q,
                                                const int update_I)
{
    using V = vec_t<T, VW>;
    const int64_t gi = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int64_t idx = gi >> lsh;
    if (idx >= ncl) return;
    const int lg = (int)(gi & ((1 << lsh) - 1));
    const int64_t c = cells[idx];
    int nb[NFM];
    bool use[NFM];
    T nsv[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = m.nbr[c * NFM + s];
        const double *g = m.geo + (c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) nsv[s][a] = (T)g[a];
        bool u = nb[s] >= 0;
        if (u && MODE != 2) {
            const int qj = m.color[nb[s]];
            u = (MODE == 0) ? (qj < q) : (qj > q);
        }
        use[s] = u;
    }
    const T base = coef[c * coef_size(D) + D + 4] + keff;
    for (int64_t qo = (int64_t)lg * VW; qo < no; qo += (int64_t)VW << lsh) {
        V nd[NFM];
#pragma unroll
        for (int s = 0; s < NFM; ++s)
            if (use[s]) nd[s] = ldv<T, VW>(dl + (int64_t)nb[s] * no + qo);
        const int64_t ix = c * no + qo;
        V ov;
        ov = ldv<T, VW>((MODE == 1 ? (const T *)dl : r) + ix);
        V dn;
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            T acc = T(0), dsum = T(0);
#pragma unroll
            for (int s = 0; s < NFM; ++s) {
                if (nb[s] == INT32_MIN) continue;
                T on = T(0);
#pragma unroll
                for (int a = 0; a < D; ++a) on += om[(qo + e) * D + a] * nsv[s][a];
                if (on > T(0))
                    dsum += on;
                else if (on < T(0) && use[s])
                    acc += on * nd[s][e];
            }
            const T dc = base + dsum * cflv_fac;
            dn[e] = (MODE == 1) ? ov[e] - acc / dc : (ov[e] - acc) / dc;
        }
        stv<T, VW>(dl + ix, dn);
        if (update_I) {
            V io;
            io = ldv<T, VW>(I + ix);
            io = io + omega * dn;
            stv<T, VW>(I + ix, io);
        }
    }
}

// ------------------------------------------------------------------ radiation: gradients, residual, sweep
template <typename T, int D, int NFM>
__global__ __launch_bounds__(256) void k_grad_I(const T *__restrict__ I, T *__restrict__ gI, const MeshDev m,
                                                const int64_t no, const int second_order,
                                                const int *__restrict__ cell_list, const int64_t ncl)
{
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & 63;
    const int64_t idx = b * 4 + (threadIdx.x >> 6);
    if (idx >= ncl) return;
    const int c = uni_i(cell_list ? cell_list[idx] : (int)idx);
    const int nfc = uni_i(m.nfc[c]);
    int nb[NFM];
    T lsq[NFM][D], dxc[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = (s < nfc) ? m.nbr[(int64_t)c * NFM + s] : -1;
        const double *g = m.geo + ((int64_t)c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            dxc[s][a] = (s < nfc) ? (T)g[D + a] : T(0);
            lsq[s][a] = (s < nfc) ? (T)g[3 * D + a] : T(0);
        }
    }
    const T eps2 = (T)m.eps2[c];
    for (int64_t q0 = 0; q0 < no; q0 += kWave) {
        const int64_t q = q0 + lane;
        if (q >= no) break;
        const T Ic = I[(int64_t)c * no + q];
        T g[D];
#pragma unroll
        for (int a = 0; a < D; ++a) g[a] = T(0);
        T dmax = T(0), dmin = T(0), mag = fabs(Ic);
#pragma unroll
        for (int s = 0; s < NFM; ++s) {
            if (nb[s] >= 0) {
                const T Ij = I[(int64_t)nb[s] * no + q], df = Ij - Ic;
                mag = fabs(Ij) > mag ? fabs(Ij) : mag;
#pragma unroll
                for (int a = 0; a < D; ++a) g[a] += lsq[s][a] * df;
                dmax = df > dmax ? df : dmax;
                dmin = df < dmin ? df : dmin;
            }
        }
        T phi = T(0);
        if (second_order) {
            phi = T(1);
            // eps^2 = (K h)^3 M^2 with M the largest |value| of the stencil, applied to the differences divided by M
                // (no underflow of the squares in FP32 where the distribution is tiny)
                const T inv = mag > tiny_val<T>() ? T(1) / mag : T(0);
#pragma unroll
            for (int s = 0; s < NFM; ++s) {
                if (s < nfc) {
                    T d2 = T(0);
#pragma unroll
                    for (int a = 0; a < D; ++a) d2 += g[a] * dxc[s][a];
                    if (d2 != T(0)) {
                        const T d1 = d2 > T(0) ? dmax : dmin;
                        const T u1 = d1 * inv, u2 = d2 * inv;
                            T p = (u1 * u1 + eps2 + T(2) * u1 * u2) / (u1 * u1 + T(2) * u2 * u2 + u1 * u2 + eps2);
                        p = p > T(1) ? T(1) : p;
                        phi = p < phi ? p : phi;
                    }
                }
            }
        }
#pragma unroll
        for (int a = 0; a < D; ++a) gI[((int64_t)c * D + a) * no + q] = phi * g[a];
    }
}

template <typename T, int D, int NFM>
__global__ __launch_bounds__(256) void k_residual_I(const T *__restrict__ I, const T *__restrict__ gI,
                                                    const T *__restrict__ coef, const T *__restrict__ om,
                                                    T *__restrict__ r, T *__restrict__ dl, T *__restrict__ Iout,
                                                    const MeshDev m, const int64_t no, const T cflv_fac,
                                                    const T omega, const T keff, const T sigR)
{
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & 63;
    const int64_t ci = b * 4 + (threadIdx.x >> 6);
    if (ci >= m.nc) return;
    const int c = uni_i((int)ci);
    const int nfc = uni_i(m.nfc[c]);
    int nb[NFM];
    T nsv[NFM][D], dxc[NFM][D], dxj[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = (s < nfc) ? m.nbr[(int64_t)c * NFM + s] : INT32_MIN;
        const double *g = m.geo + ((int64_t)c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            nsv[s][a] = (s < nfc) ? (T)g[a] : T(0);
            dxc[s][a] = (s < nfc) ? (T)g[D + a] : T(0);
            dxj[s][a] = (s < nfc) ? (T)g[2 * D + a] : T(0);
        }
    }
    const T B = coef[(int64_t)c * coef_size(D) + D + 3];
    const T inv_dtR = coef[(int64_t)c * coef_size(D) + D + 4];
    for (int64_t q0 = 0; q0 < no; q0 += kWave) {
        const int64_t q = q0 + lane;
        if (q >= no) break;
        T o[D];
#pragma unroll
        for (int a = 0; a < D; ++a) o[a] = om[q * D + a];
        const T Ic = I[(int64_t)c * no + q];
        T gc[D];
#pragma unroll
        for (int a = 0; a < D; ++a) gc[a] = gI[((int64_t)c * D + a) * no + q];
        T flux = T(0), dsum = T(0);
#pragma unroll
        for (int s = 0; s < NFM; ++s) {
            if (nb[s] == INT32_MIN) continue;
            T on = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) on += o[a] * nsv[s][a];
            T Iv;
            if (on > T(0)) {
                Iv = Ic;
#pragma unroll
                for (int a = 0; a < D; ++a) Iv += gc[a] * dxc[s][a];
                dsum += on;
            } else if (nb[s] >= 0) {
                const int64_t j = nb[s];
                Iv = I[j * no + q];
#pragma unroll
                for (int a = 0; a < D; ++a) Iv += gI[(j * D + a) * no + q] * dxj[s][a];
            } else {
                const T Tb = (T)m.bcs[m.bf_tag[-nb[s] - 1]].T;
                Iv = sigR * Tb * Tb * Tb * Tb / T(kPi);
            }
            flux += on * Iv;
        }
        const T rr = keff * (B - Ic) - flux;
        const T dcoef = inv_dtR + keff + dsum * cflv_fac;
        const int64_t idx = (int64_t)c * no + q;
        if (Iout) {
            Iout[idx] = Ic + omega * (rr / dcoef);
        } else {
            r[idx] = rr;
            if (dl) dl[idx] = rr / dcoef;
        }
    }
}

template <typename T, int D, int NFM>
__global__ __launch_bounds__(256) void k_sweep_I(const T *__restrict__ r, const T *__restrict__ dlin,
                                                 T *__restrict__ dlout, const T *__restrict__ I,
                                                 T *__restrict__ Iout, const T *__restrict__ coef,
                                                 const T *__restrict__ om, const MeshDev m, const int64_t no,
                                                 const T cflv_fac, const T omega, const T keff)
{
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & 63;
    const int64_t ci = b * 4 + (threadIdx.x >> 6);
    if (ci >= m.nc) return;
    const int c = uni_i((int)ci);
    const int nfc = uni_i(m.nfc[c]);
    int nb[NFM];
    T nsv[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = (s < nfc) ? m.nbr[(int64_t)c * NFM + s] : INT32_MIN;
        const double *g = m.geo + ((int64_t)c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) nsv[s][a] = (s < nfc) ? (T)g[a] : T(0);
    }
    const T base = coef[(int64_t)c * coef_size(D) + D + 4] + keff;
    for (int64_t q0 = 0; q0 < no; q0 += kWave) {
        const int64_t q = q0 + lane;
        if (q >= no) break;
        T acc = T(0), dsum = T(0);
#pragma unroll
        for (int s = 0; s < NFM; ++s) {
            if (nb[s] == INT32_MIN) continue;
            T on = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) on += om[q * D + a] * nsv[s][a];
            if (on > T(0))
                dsum += on;
            else if (on < T(0) && nb[s] >= 0)
                acc += on * dlin[(int64_t)nb[s] * no + q];
        }
        const int64_t idx = (int64_t)c * no + q;
        const T dn = (r[idx] - acc) / (base + dsum * cflv_fac);
        if (Iout)
            Iout[idx] = I[idx] + omega * dn;
        else
            dlout[idx] = dn;
    }
}

// Packed vector forms of the ordinate kernels for N_o divisible by VW: a cell's ordinates are spread over
// 2^lsh consecutive lanes (the smallest power of two covering N_o / VW, at most 64), so one wave serves
// 64 >> lsh cells; each lane owns VW consecutive ordinates (one 16-byte access per row).  Per-cell
// tables are loaded per lane (the lanes of a cell read the same addresses).  Same arithmetic as the
// scalar kernels.
template <typename T, int D, int NFM, int VW>
__global__ __launch_bounds__(256) void k_grad_Iv(const T *__restrict__ I, T *__restrict__ gI, const MeshDev m,
                                                 const int64_t no, const int lsh, const int second_order,
                                                 const int *__restrict__ cell_list, const int64_t ncl)
{
    using V = vec_t<T, VW>;
    const int64_t gi = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int64_t idx = gi >> lsh;
    if (idx >= ncl) return;
    const int lg = (int)(gi & ((1 << lsh) - 1));
    const int64_t c = cell_list ? cell_list[idx] : idx;
    int nb[NFM];
    T lsq[NFM][D], dxc[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = m.nbr[c * NFM + s];
        const double *g = m.geo + (c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            dxc[s][a] = (T)g[D + a];
            lsq[s][a] = (T)g[3 * D + a];
        }
    }
    const T eps2 = (T)m.eps2[c];
    for (int64_t q = (int64_t)lg * VW; q < no; q += (int64_t)VW << lsh) {
        const V Ic = *(const V *)(I + c * no + q);
        V nbv[NFM];
#pragma unroll
        for (int s = 0; s < NFM; ++s)
            if (nb[s] >= 0) nbv[s] = *(const V *)(I + (int64_t)nb[s] * no + q);
        V go[D];
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            T g[D];
#pragma unroll
            for (int a = 0; a < D; ++a) g[a] = T(0);
            T dmax = T(0), dmin = T(0), mag = fabs(Ic[e]);
#pragma unroll
            for (int s = 0; s < NFM; ++s) {
                if (nb[s] >= 0) {
                    const T Ij = nbv[s][e], df = Ij - Ic[e];
                    mag = fabs(Ij) > mag ? fabs(Ij) : mag;
#pragma unroll
                    for (int a = 0; a < D; ++a) g[a] += lsq[s][a] * df;
                    dmax = df > dmax ? df : dmax;
                    dmin = df < dmin ? df : dmin;
                }
            }
            T phi = T(0);
            if (second_order) {
                phi = T(1);
                // eps^2 = (K h)^3 M^2 with M the largest |value| of the stencil, applied to the differences divided by M
                // (no underflow of the squares in FP32 where the distribution is tiny)
                const T inv = mag > tiny_val<T>() ? T(1) / mag : T(0);
#pragma unroll
                for (int s = 0; s < NFM; ++s) {
                    if (nb[s] != INT32_MIN) {
                        T d2 = T(0);
#pragma unroll
                        for (int a = 0; a < D; ++a) d2 += g[a] * dxc[s][a];
                        if (d2 != T(0)) {
                            const T d1 = d2 > T(0) ? dmax : dmin;
                            const T u1 = d1 * inv, u2 = d2 * inv;
                            T p = (u1 * u1 + eps2 + T(2) * u1 * u2) / (u1 * u1 + T(2) * u2 * u2 + u1 * u2 + eps2);
                            p = p > T(1) ? T(1) : p;
                            phi = p < phi ? p : phi;
                        }
                    }
                }
            }
#pragma unroll
            for (int a = 0; a < D; ++a) go[a][e] = phi * g[a];
        }
#pragma unroll
        for (int a = 0; a < D; ++a) *(V *)(gI + (c * D + a) * no + q) = go[a];
    }
}

template <typename T, int D, int NFM, int VW>
__global__ __launch_bounds__(256) void k_residual_Iv(const T *__restrict__ I, const T *__restrict__ gI,
                                                     const T *__restrict__ coef, const T *__restrict__ om,
                                                     T *__restrict__ r, T *__restrict__ dl, T *__restrict__ Iout,
                                                     const MeshDev m, const int64_t no, const int lsh,
                                                     const T cflv_fac, const T omega, const T keff, const T sigR)
{
    using V = vec_t<T, VW>;
    const int64_t gi = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int64_t c = gi >> lsh;
    if (c >= m.nc) return;
    const int lg = (int)(gi & ((1 << lsh) - 1));
    int nb[NFM];
    T nsv[NFM][D], dxc[NFM][D], dxj[NFM][D], Tb4[NFM];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = m.nbr[c * NFM + s];
        const double *g = m.geo + (c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            nsv[s][a] = (T)g[a];
            dxc[s][a] = (T)g[D + a];
            dxj[s][a] = (T)g[2 * D + a];
        }
        Tb4[s] = T(0);
        if (nb[s] < 0 && nb[s] != INT32_MIN) {
            const T Tb = (T)m.bcs[m.bf_tag[-nb[s] - 1]].T;
            Tb4[s] = sigR * Tb * Tb * Tb * Tb / T(kPi);
        }
    }
    const T B = coef[c * coef_size(D) + D + 3];
    const T inv_dtR = coef[c * coef_size(D) + D + 4];
    for (int64_t q = (int64_t)lg * VW; q < no; q += (int64_t)VW << lsh) {
        const V Ic = *(const V *)(I + c * no + q);
        V gc[D];
#pragma unroll
        for (int a = 0; a < D; ++a) gc[a] = *(const V *)(gI + (c * D + a) * no + q);
        V nI[NFM], ng[NFM][D];
#pragma unroll
        for (int s = 0; s < NFM; ++s)
            if (nb[s] >= 0) {
                nI[s] = *(const V *)(I + (int64_t)nb[s] * no + q);
#pragma unroll
                for (int a = 0; a < D; ++a) ng[s][a] = *(const V *)(gI + ((int64_t)nb[s] * D + a) * no + q);
            }
        V rr, dd;
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            T o[D];
#pragma unroll
            for (int a = 0; a < D; ++a) o[a] = om[(q + e) * D + a];
            T flux = T(0), dsum = T(0);
#pragma unroll
            for (int s = 0; s < NFM; ++s) {
                if (nb[s] == INT32_MIN) continue;
                T on = T(0);
#pragma unroll
                for (int a = 0; a < D; ++a) on += o[a] * nsv[s][a];
                T Iv;
                if (on > T(0)) {
                    Iv = Ic[e];
#pragma unroll
                    for (int a = 0; a < D; ++a) Iv += gc[a][e] * dxc[s][a];
                    dsum += on;
                } else if (nb[s] >= 0) {
                    Iv = nI[s][e];
#pragma unroll
                    for (int a = 0; a < D; ++a) Iv += ng[s][a][e] * dxj[s][a];
                } else {
                    Iv = Tb4[s];
                }
                flux += on * Iv;
            }
            rr[e] = keff * (B - Ic[e]) - flux;
            dd[e] = inv_dtR + keff + dsum * cflv_fac;
        }
        const int64_t idx = c * no + q;
        if (Iout) {
            *(V *)(Iout + idx) = Ic + omega * (rr / dd);
        } else {
            *(V *)(r + idx) = rr;
            if (dl) *(V *)(dl + idx) = rr / dd;
        }
    }
}

template <typename T, int D, int NFM, int VW>
__global__ __launch_bounds__(256) void k_sweep_Iv(const T *__restrict__ r, const T *__restrict__ dlin,
                                                  T *__restrict__ dlout, const T *__restrict__ I,
                                                  T *__restrict__ Iout, const T *__restrict__ coef,
                                                  const T *__restrict__ om, const MeshDev m, const int64_t no,
                                                  const int lsh, const T cflv_fac, const T omega, const T keff)
{
    using V = vec_t<T, VW>;
    const int64_t gi = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const int64_t c = gi >> lsh;
    if (c >= m.nc) return;
    const int lg = (int)(gi & ((1 << lsh) - 1));
    int nb[NFM];
    T nsv[NFM][D];
#pragma unroll
    for (int s = 0; s < NFM; ++s) {
        nb[s] = m.nbr[c * NFM + s];
        const double *g = m.geo + (c * NFM + s) * 4 * D;
#pragma unroll
        for (int a = 0; a < D; ++a) nsv[s][a] = (T)g[a];
    }
    const T base = coef[c * coef_size(D) + D + 4] + keff;
    for (int64_t q = (int64_t)lg * VW; q < no; q += (int64_t)VW << lsh) {
        V nd[NFM];
#pragma unroll
        for (int s = 0; s < NFM; ++s)
            if (nb[s] >= 0) nd[s] = *(const V *)(dlin + (int64_t)nb[s] * no + q);
        const int64_t idx = c * no + q;
        const V rv = *(const V *)(r + idx);
        V dn;
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            T acc = T(0), dsum = T(0);
#pragma unroll
            for (int s = 0; s < NFM; ++s) {
                if (nb[s] == INT32_MIN) continue;
                T on = T(0);
#pragma unroll
                for (int a = 0; a < D; ++a) on += om[(q + e) * D + a] * nsv[s][a];
                if (on > T(0))
                    dsum += on;
                else if (on < T(0) && nb[s] >= 0)
                    acc += on * nd[s][e];
            }
            dn[e] = (rv[e] - acc) / (base + dsum * cflv_fac);
        }
        if (Iout)
            *(V *)(Iout + idx) = *(const V *)(I + idx) + omega * dn;
        else
            *(V *)(dlout + idx) = dn;
    }
}

// ------------------------------------------------------------------ moments (Eq. getmoment, reduced form)
// Raw FP64 moments about a reference velocity u_ref (the cell's previous velocity) reduced across the
// wave, then shifted to central moments.  mom layout: see MomLayout.
template <typename T, int D, int VW>
__global__ __launch_bounds__(256) void k_moments(const T *__restrict__ f, const T *__restrict__ I,
                                                 const double *__restrict__ xi, const double *__restrict__ w,
                                                 const double *__restrict__ om, const double *__restrict__ wo,
                                                 const double *__restrict__ uref, double *__restrict__ mom,
                                                 const int64_t nc, const int64_t nv, const int64_t no,
                                                 const double dr, const double dv, const double Tvref)
{
    constexpr int ND = (D == 3) ? 3 : 4;
    constexpr MomLayout L{D};
    // kMomLanes lanes per cell, 16 cells per block: the four cells of a wave share each load of the
    // velocity nodes and weights, and one butterfly step of the final sums serves all four
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & (kMomLanes - 1);
    const int64_t ci = b * (256 / kMomLanes) + (threadIdx.x / kMomLanes);
    const bool valid = ci < nc;
    const int64_t c = valid ? ci : nc - 1;  // clamped: the group runs, only its store is skipped
    double ur[D];
#pragma unroll
    for (int a = 0; a < D; ++a) ur[a] = uref ? uref[(int64_t)c * L.size() + L.u() + a] : 0.0;
    // accumulators: G: m0, m1[D], m2[D*D], m3[D]; H: h0, h1[D]; R: r0, r1[D]; V: v0, v1[D]
    double m0 = 0, m1[D], m2[D][D], m3[D], h0 = 0, h1[D], r0 = 0, r1[D], v0 = 0, v1[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        m1[a] = m3[a] = h1[a] = r1[a] = v1[a] = 0;
#pragma unroll
        for (int bb = 0; bb < D; ++bb) m2[a][bb] = 0;
    }
#pragma unroll 4
    for (int64_t kb = (int64_t)lane * VW; kb < nv; kb += kMomLanes * VW) {
      T fG[VW], fR[VW], fV[VW], fH[VW];
      load_vw_nt<T, VW>(f + (c * ND + 0) * nv + kb, fG);
      load_vw_nt<T, VW>(f + (c * ND + 1) * nv + kb, fR);
      load_vw_nt<T, VW>(f + (c * ND + 2) * nv + kb, fV);
      if (ND == 4) load_vw_nt<T, VW>(f + (c * ND + (ND == 4 ? 3 : 0)) * nv + kb, fH);
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const int64_t k = kb + e;
        if (VW == 1 && k >= nv) break;
        const double wk = w[k];
        double cc[D], c2 = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            cc[a] = xi[k * D + a] - ur[a];
            c2 += cc[a] * cc[a];
        }
        const double G = wk * (double)fG[e];
        const double R = wk * (double)fR[e];
        const double V = wk * (double)fV[e];
        const double H = (ND == 4) ? wk * (double)fH[e] : 0.0;
        m0 += G;
        h0 += H;
        r0 += R;
        v0 += V;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double cG = cc[a] * G;
            m1[a] += cG;
            m3[a] += cG * c2;
            h1[a] += cc[a] * H;
            r1[a] += cc[a] * R;
            v1[a] += cc[a] * V;
            // the second moment is symmetric: its upper triangle, mirrored after the sums
#pragma unroll
            for (int bb = a; bb < D; ++bb) m2[a][bb] += cc[bb] * cG;
        }
      }
    }
    m0 = group_sum<kMomLanes>(m0);
    h0 = group_sum<kMomLanes>(h0);
    r0 = group_sum<kMomLanes>(r0);
    v0 = group_sum<kMomLanes>(v0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        m1[a] = group_sum<kMomLanes>(m1[a]);
        m3[a] = group_sum<kMomLanes>(m3[a]);
        h1[a] = group_sum<kMomLanes>(h1[a]);
        r1[a] = group_sum<kMomLanes>(r1[a]);
        v1[a] = group_sum<kMomLanes>(v1[a]);
#pragma unroll
        for (int bb = a; bb < D; ++bb) m2[a][bb] = group_sum<kMomLanes>(m2[a][bb]);
    }
#pragma unroll
    for (int a = 1; a < D; ++a)
#pragma unroll
        for (int bb = 0; bb < a; ++bb) m2[a][bb] = m2[bb][a];
    double eR = 0, qR[D];
#pragma unroll
    for (int a = 0; a < D; ++a) qR[a] = 0;
    for (int64_t q = lane; q < no; q += kMomLanes) {
        const double Iq = wo[q] * (double)I[c * no + q];
        eR += Iq;
#pragma unroll
        for (int a = 0; a < D; ++a) qR[a] += om[q * D + a] * Iq;
    }
    eR = group_sum<kMomLanes>(eR);
#pragma unroll
    for (int a = 0; a < D; ++a) qR[a] = group_sum<kMomLanes>(qR[a]);
    if (lane == 0 && valid) {
        double *M = mom + c * L.size();
        const double rho = m0;
        double dl[D], d2 = 0, S2 = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            dl[a] = m1[a] / rho;
            d2 += dl[a] * dl[a];
            S2 += m2[a][a];
        }
        const double Tt = (S2 - rho * d2 + h0) / (3.0 * rho);
        M[L.rho()] = rho;
#pragma unroll
        for (int a = 0; a < D; ++a) M[L.u() + a] = ur[a] + dl[a];
        M[L.Tt()] = Tt;
        M[L.Tr()] = 2.0 * r0 / (dr * rho);
        M[L.Tv()] = Tvref > 0 ? Tvref / log1p(Tvref * rho / v0) : 2.0 * v0 / (dv * rho);
        M[L.eR()] = eR;
        M[L.er()] = r0;
        M[L.ev()] = v0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
#pragma unroll
            for (int bb = 0; bb < D; ++bb)
                M[L.sig() + a * D + bb] = m2[a][bb] - rho * dl[a] * dl[bb] - (a == bb ? rho * Tt : 0.0);
            double t3 = m3[a] - dl[a] * S2 + 2.0 * rho * dl[a] * d2;
#pragma unroll
            for (int bb = 0; bb < D; ++bb) t3 -= 2.0 * dl[bb] * m2[a][bb];
            M[L.qt() + a] = 0.5 * (t3 + h1[a] - dl[a] * h0);
            M[L.qr() + a] = r1[a] - dl[a] * r0;
            M[L.qv() + a] = v1[a] - dl[a] * v0;
            M[L.qR() + a] = qR[a];
        }
    }
}

// ------------------------------------------------------------------ per-cell coefficients (prologue)
template <typename T, int D>
__global__ void k_prologue(const double *__restrict__ mom, T *__restrict__ coef, const double *__restrict__ h,
                           const int64_t nc, const Phys p, const double cfl_meso)
{
    constexpr MomLayout L{D};
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double *M = mom + c * L.size();
    T *cf = coef + c * coef_size(D);
    const double rho = M[L.rho()], Tt = M[L.Tt()], Tr = M[L.Tr()], Tv = M[L.Tv()], eR = M[L.eR()];
    const double Ttr = (3 * Tt + p.d_r * Tr) / (3 + p.d_r), Ttv = vib_Ttv(p, Tt, Tv);
    const double tau = sqrt(2.0 / kPi) * pow(Tt, p.omega - 1.0) * p.Kn / rho;
    double qt[3] = {0, 0, 0}, qr[3] = {0, 0, 0}, qv[3] = {0, 0, 0}, q0[3], q1[3], q2[3];
    double un = 0;
    for (int a = 0; a < D; ++a) {
        qt[a] = M[L.qt() + a];
        qr[a] = M[L.qr() + a];
        qv[a] = M[L.qv() + a];
        cf[a] = (T)M[L.u() + a];
        un += M[L.u() + a] * M[L.u() + a];
    }
    for (int a = 0; a < 3; ++a) {
        q0[a] = p.Q[0][0] * qt[a] + p.Q[0][1] * qr[a] + p.Q[0][2] * qv[a];
        q1[a] = p.Q[1][0] * qt[a] + p.Q[1][1] * qr[a] + p.Q[1][2] * qv[a];
        q2[a] = p.Q[2][0] * qt[a] + p.Q[2][1] * qr[a] + p.Q[2][2] * qv[a];
    }
    const double cs = sqrt(5.0 / 3.0 * Tt);
    const double Tv4 = Tv * Tv * Tv * Tv;
    cf[D] = (T)(1.0 / tau);
    cf[D + 1] = (T)((sqrt(un) + cs) / (cfl_meso * h[c]));
    cf[D + 2] = (T)(p.keff * (4 * p.sigma_R * Tv4 - eR) / rho);
    cf[D + 3] = (T)(p.sigma_R * Tv4 / kPi);
    cf[D + 4] = (T)(1.0 / (cfl_meso * h[c]));
    // point-implicit rate of the emission part of the gas-photon exchange on f2: d(k_eff e_vR) / d(rho e_v),
    // 4 k_eff e_vR / e_v with a constant d_v, 4 k_eff e_vR / (rho T_v c_v(T_v)) with d_v(T)
    cf[D + 5] = (T)(p.Tvref > 0 ? 4.0 * p.keff * 4 * p.sigma_R * Tv4 / (rho * Tv * vib_cv(p, Tv))
                                : 4.0 * p.keff * 4 * p.sigma_R * Tv4 / M[L.ev()]);
    const double TX[3] = {Tt, Ttr, Ttv};
    const double *qX[3] = {qt, q0, q0};
    const double TRX[3] = {Tr, Ttr, Tr};
    const double *qRX[3] = {qr, q1, q1};
    const double TVX[3] = {Tv, Tv, Ttv};
    // e_v(T_v) (g_2t, g_2r) and e_v(T_tv) (g_2v): d_v(T) T / 2
    const double EVX[3] = {vib_e(p, Tv), vib_e(p, Tv), vib_e(p, Ttv)};
    const double *qVX[3] = {qv, q2, q2};
    for (int X = 0; X < 3; ++X) {
        T *px = cf + D + 6 + X * coef_x(D);
        const double T_ = TX[X];
        px[0] = (T)(1.0 / (2.0 * T_));
        px[1] = (T)(rho * pow(2.0 * kPi * T_, -0.5 * D));
        for (int a = 0; a < D; ++a) {
            px[2 + a] = (T)(2.0 * qX[X][a] / (15.0 * T_ * rho * T_));
            px[3 + D + a] = (T)(qRX[X][a] / (T_ * rho));
            px[4 + 2 * D + a] = (T)(qVX[X][a] / (T_ * rho));
        }
        px[2 + D] = (T)(0.5 * p.d_r * TRX[X]);
        px[3 + 2 * D] = (T)(p.Tvref > 0 ? EVX[X] : 0.5 * p.d_v * TVX[X]);
        px[4 + 3 * D] = (T)((3 - D) * T_);
    }
}

// ------------------------------------------------------------------ discrete-conservative corrections
// Per cell (one wave, lanes over the velocities): for each reference temperature X the discrete sums of the
// reference distributions exactly as collision() evaluates them (T precision, FP64 accumulation) -- the
// normal matrix B = sum w psi psi^T e with psi = (1, c, c^2/2), e = rho f0^eq(T_X), the moments sum w psi G
// and the densities of R, V, H -- then, on the first lane, the correction whose discrete moments restore
// (rho, 0, (D/2) rho T_X) for G and (d_r/2) T_RX rho, e_v(T_VX) rho, (3 - D) T_X rho for R, V, H.  The
// normal equations are solved by Cholesky; a pivot below 1e-12 of its diagonal leaves G uncorrected.
__device__ inline bool chol_solve(const int n, double (&A)[5][5], double (&b)[5])
{
    double L[5][5];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = A[i][j];
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            if (i != j) {
                L[i][j] = v / L[j][j];
            } else if (v > 1e-12 * A[i][i]) {
                L[i][i] = sqrt(v);
            } else {
                return false;
            }
        }
    for (int i = 0; i < n; ++i) {  // forward substitution, in place
        for (int k = 0; k < i; ++k) b[i] -= L[i][k] * b[k];
        b[i] /= L[i][i];
    }
    for (int i = n - 1; i >= 0; --i) {  // back substitution
        for (int k = i + 1; k < n; ++k) b[i] -= L[k][i] * b[k];
        b[i] /= L[i][i];
    }
    return true;
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_cons_sums(const double *__restrict__ mom, const T *__restrict__ coef,
                                                   const T *__restrict__ xi, const double *__restrict__ w,
                                                   T *__restrict__ ccons, const int64_t nc, const int64_t nv,
                                                   const Phys p)
{
    constexpr MomLayout L{D};
    constexpr int n = D + 2, NB = (D + 2) * (D + 3) / 2;
    const int64_t c = xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= nc) return;
    const T *cf = coef + c * coef_size(D);
    const double *M = mom + c * L.size();
    const double rho = M[L.rho()], Tt = M[L.Tt()], Tr = M[L.Tr()], Tv = M[L.Tv()];
    const double Ttr = (3 * Tt + p.d_r * Tr) / (3 + p.d_r), Ttv = vib_Ttv(p, Tt, Tv);
    const double TX[3] = {Tt, Ttr, Ttv}, TRX[3] = {Tr, Ttr, Tr};
    const double VX[3] = {p.Tvref > 0 ? vib_e(p, Tv) : 0.5 * p.d_v * Tv, p.Tvref > 0 ? vib_e(p, Tv) : 0.5 * p.d_v * Tv,
                          p.Tvref > 0 ? vib_e(p, Ttv) : 0.5 * p.d_v * Ttv};
    T *out = ccons + c * 3 * kConsX;
    const T aG = T(0.5) * T(2 + D), aH = T(0.5) * T(D);
    for (int X = 0; X < 3; ++X) {
        const T *px = cf + D + 6 + X * coef_x(D);
        double sB[NB], sG[n], sR = 0, sV = 0, sH = 0;
        for (int i = 0; i < NB; ++i) sB[i] = 0;
        for (int i = 0; i < n; ++i) sG[i] = 0;
        for (int64_t k = lane; k < nv; k += kWave) {
            T cc[D], c2 = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                cc[a] = xi[k * D + a] - cf[a];
                c2 += cc[a] * cc[a];
            }
            const T e = px[1] * dexp<T>(-c2 * px[0]);
            T s = T(0), br = T(0), bv = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                s += px[2 + a] * cc[a];
                br += px[3 + D + a] * cc[a];
                bv += px[4 + 2 * D + a] * cc[a];
            }
            const T q = c2 * px[0];
            const T G = e * (T(1) + s * (q - aG));
            const double wk = w[k];
            double psi[n];
            psi[0] = 1.0;
#pragma unroll
            for (int a = 0; a < D; ++a) psi[1 + a] = (double)cc[a];
            psi[D + 1] = 0.5 * (double)c2;
            int ib = 0;
#pragma unroll
            for (int i = 0; i < n; ++i) {
                sG[i] += wk * psi[i] * (double)G;
#pragma unroll
                for (int j = 0; j <= i; ++j) sB[ib++] += wk * psi[i] * psi[j] * (double)e;
            }
            sR += wk * (double)(px[2 + D] * G + br * e);
            sV += wk * (double)(px[3 + 2 * D] * G + bv * e);
            if (D < 3) sH += wk * (double)(px[4 + 3 * D] * e * (T(1) + s * (q - aH)));
        }
        for (int i = 0; i < NB; ++i) sB[i] = wave_sum(sB[i]);
        for (int i = 0; i < n; ++i) sG[i] = wave_sum(sG[i]);
        sR = wave_sum(sR);
        sV = wave_sum(sV);
        sH = wave_sum(sH);
        if (lane == 0) {
            double A[5][5], b[5];
            int ib = 0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j <= i; ++j) A[i][j] = A[j][i] = sB[ib++];
            for (int i = 0; i < n; ++i) b[i] = -sG[i];
            b[0] += rho;
            b[D + 1] += 0.5 * D * rho * TX[X];
            T *o = out + X * kConsX;
            for (int i = 0; i < kConsX; ++i) o[i] = T(0);
            if (chol_solve(n, A, b)) {
                o[0] = (T)b[0];
                o[1] = (T)(b[D + 1] * TX[X]);
                for (int a = 0; a < D; ++a) o[2 + a] = (T)b[1 + a];
            }
            const double S = sB[0];
            o[D + 2] = (T)((0.5 * p.d_r * TRX[X] * rho - sR) / S);
            o[D + 3] = (T)((VX[X] * rho - sV) / S);
            o[D + 4] = (T)(D < 3 ? ((3 - D) * TX[X] * rho - sH) / S : 0.0);
        }
    }
}

template <typename T, int D>
void launch_cons_sums(const double *mom, const T *coef, const T *xi, const double *w, T *ccons, int64_t nc,
                      int64_t nv, const Phys &p, hipStream_t st)
{
    hipLaunchKernelGGL((k_cons_sums<T, D>), dim3((unsigned)((nc + 3) / 4)), dim3(256), 0, st, mom, coef, xi, w, ccons,
                       nc, nv, p);
}

// ------------------------------------------------------------------ wall re-emission densities
// Wall density of each diffuse-wall face (zero net mass flux): outgoing flux of the reconstructed f over
// the incoming flux of the unit-density wall Maxwellian.  One 256-thread block per boundary face; the
// loop body is branch-free (both sides evaluated, the sign of xi.n selects), so the loads of several
// velocities are in flight together.
template <typename T, int D, int NFM>
__global__ __launch_bounds__(256) void k_wall_density(const T *__restrict__ f, const T *__restrict__ gf,
                                                      const int *__restrict__ grow, const double *__restrict__ xi,
                                                      const double *__restrict__ w, T *__restrict__ rhow,
                                                      const MeshDev m, const int64_t nv)
{
    constexpr int ND = (D == 3) ? 3 : 4;
    __shared__ double sh[2][4];
    const int bfi = blockIdx.x;
    const int t = threadIdx.x;
    const BcDev bc = m.bf_bc[bfi];
    if (bc.kind != 0) {
        if (t == 0) rhow[bfi] = (T)0;
        return;
    }
    const int64_t c = m.bf_cell[bfi], cg = grow[bfi];  // cg: the cell's row in gf
    double n[D], dx[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        n[a] = m.bf_n[(int64_t)bfi * D + a];
        dx[a] = m.bf_dxc[(int64_t)bfi * D + a];
    }
    const double gn = gauss_norm<D>(1.0, bc.T);
    double out = 0, in = 0;
#pragma unroll 4
    for (int64_t k = t; k < nv; k += 256) {
        double xn = 0, c2 = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            xn += xi[k * D + a] * n[a];
            const double cc = xi[k * D + a] - bc.u[a];
            c2 += cc * cc;
        }
        T v = f[(c * ND + 0) * nv + k];
#pragma unroll
        for (int a = 0; a < D; ++a) v += gf[((cg * ND + 0) * D + a) * nv + k] * (T)dx[a];
        const double mw = w[k] * (-xn) * gn * exp(-c2 / (2 * bc.T));
        if (xn > 0) out += w[k] * xn * (double)v;
        else in += mw;
    }
    out = block4_sum(out, sh[0]);
    in = block4_sum(in, sh[1]);
    if (t == 0) rhow[bfi] = (T)(out / in);
}

// ------------------------------------------------------------------ boundary flux moments of a state
// per boundary face: NW outward fluxes (mass, momentum D, total energy, e_r, e_v, e_R) per unit area and
// the surface output (q_conv, q_rad, p_w)
template <typename T, int D>
__global__ __launch_bounds__(256) void k_boundary_flux(const T *__restrict__ f, const T *__restrict__ gf,
                                                       const int *__restrict__ grow,
                                                       const T *__restrict__ I, const T *__restrict__ gI,
                                                       const double *__restrict__ xi, const double *__restrict__ w,
                                                       const double *__restrict__ om, const double *__restrict__ wo,
                                                       const T *__restrict__ rhow, double *__restrict__ bflux,
                                                       double *__restrict__ bsurf, const MeshDev m, const int64_t nv,
                                                       const int64_t no, const double dr, const double dv,
                                                       const double sigR)
{
    constexpr int ND = (D == 3) ? 3 : 4;
    constexpr int NW = D + 5;
    __shared__ double sh[NW + 3][4];
    const int bfi = blockIdx.x;
    const int t = threadIdx.x;
    const BcDev bc = m.bf_bc[bfi];
    const int64_t c = m.bf_cell[bfi], cg = grow[bfi];  // cg: the cell's row in gf
    double n[D], dx[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        n[a] = m.bf_n[(int64_t)bfi * D + a];
        dx[a] = m.bf_dxc[(int64_t)bfi * D + a];
    }
    const double rho_in = (bc.kind == 0) ? (double)rhow[bfi] : bc.rho;
    const double gn = gauss_norm<D>(rho_in, bc.T);
    double F[NW], qconv = 0, pw = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) F[i] = 0;
    // branch-free body (both sides evaluated, the sign of xi.n selects) so that the loads of several
    // velocities are in flight together
#pragma unroll 2
    for (int64_t k = t; k < nv; k += 256) {
        double x[D], xn = 0, x2 = 0, c2 = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            x[a] = xi[k * D + a];
            xn += x[a] * n[a];
            x2 += x[a] * x[a];
            c2 += (x[a] - bc.u[a]) * (x[a] - bc.u[a]);
        }
        double fo[4] = {0, 0, 0, 0};
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            T v = f[(c * ND + d) * nv + k];
#pragma unroll
            for (int a = 0; a < D; ++a) v += gf[((cg * ND + d) * D + a) * nv + k] * (T)dx[a];
            fo[d] = (double)v;
        }
        const double G = gn * exp(-c2 / (2 * bc.T));
        double fv[4];
        if (xn > 0) {
            fv[0] = fo[0];
            fv[1] = fo[1];
            fv[2] = fo[2];
            fv[3] = fo[3];
        } else {
            fv[0] = G;
            fv[1] = 0.5 * dr * bc.T * G;
            fv[2] = bc.ev * G;
            fv[3] = (3 - D) * bc.T * G;
        }
        const double wk = w[k];
        const double hv = (ND == 4) ? fv[3] : 0.0;
        const double en = 0.5 * x2 * fv[0] + 0.5 * hv + fv[1] + fv[2];
        F[0] += wk * xn * fv[0];
#pragma unroll
        for (int a = 0; a < D; ++a) F[1 + a] += wk * xn * x[a] * fv[0];
        F[D + 1] += wk * xn * en;
        F[D + 2] += wk * xn * fv[1];
        F[D + 3] += wk * xn * fv[2];
        qconv += wk * xn * en;
        pw += wk * xn * xn * fv[0];
    }
    double qrad = 0;
    for (int64_t q = t; q < no; q += 256) {
        double on = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) on += om[q * D + a] * n[a];
        double Iv;
        if (on > 0) {
            T v = I[c * no + q];
#pragma unroll
            for (int a = 0; a < D; ++a) v += gI[(c * D + a) * no + q] * (T)dx[a];
            Iv = (double)v;
        } else {
            Iv = sigR * bc.T * bc.T * bc.T * bc.T / kPi;
        }
        qrad += wo[q] * on * Iv;
    }
#pragma unroll
    for (int i = 0; i < NW; ++i) F[i] = block4_sum(F[i], sh[i]);
    qconv = block4_sum(qconv, sh[NW]);
    pw = block4_sum(pw, sh[NW + 1]);
    qrad = block4_sum(qrad, sh[NW + 2]);
    if (t == 0) {
        double *out = bflux + (int64_t)bfi * NW;
        for (int i = 0; i < NW; ++i) out[i] = F[i];
        out[D + 4] = qrad;
        out[D + 1] += qrad;
        bsurf[(int64_t)bfi * 3 + 0] = qconv;
        bsurf[(int64_t)bfi * 3 + 1] = qrad;
        bsurf[(int64_t)bfi * 3 + 2] = pw;
    }
}

// ------------------------------------------------------------------ synchronisation and initialisation
// f += f^eq(M1) - f^eq(M0) with f^eq the multi-temperature equilibrium; I += (eR1 - eR0)/(4 pi).
// sp per cell: [rho, u[D], Tt, Tr, Tv, eR] for M0 then M1.
template <typename T, int D, int VW>
__global__ __launch_bounds__(256) void k_sync(T *__restrict__ f, T *__restrict__ I, const double *__restrict__ sp,
                                              const double *__restrict__ xi, const int64_t nc, const int64_t nv,
                                              const int nchunk, const int cgroup, const int64_t no,
                                              const double dr, const double dv, const double Tvref,
                                              const int init)
{
    constexpr int ND = (D == 3) ? 3 : 4;
    constexpr int NS = D + 5;
    // one wave per (cell, chunk of kWave * VW velocities); chunk 0 also updates the cell's ordinates
    const int lane = threadIdx.x & 63;
    const int w = uni_i((int)(xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6)));
    int c, ch;
    if (!wave_cell_chunk(w, (int)nc, nchunk, cgroup, c, ch)) return;
    const double *s0 = sp + (int64_t)c * 2 * NS, *s1 = s0 + NS;
    const double n0 = gauss_norm<D>(s0[0], s0[D + 1]), n1 = gauss_norm<D>(s1[0], s1[D + 1]);
    // e_v(T_v) of the two states (variable d_v)
    const double ev0 = Tvref > 0 ? Tvref / expm1(Tvref / s0[D + 3]) : 0.0;
    const double ev1 = Tvref > 0 ? Tvref / expm1(Tvref / s1[D + 3]) : 0.0;
    const int64_t kb = ((int64_t)ch * kWave + lane) * VW;
    if (kb < nv) {
      T fv[4][VW];
      if (!init) {
#pragma unroll
        for (int d = 0; d < ND; ++d) load_vw_nt<T, VW>(f + ((int64_t)c * ND + d) * nv + kb, fv[d]);
      }
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const int64_t k = kb + e;
        double c20 = 0, c21 = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double x = xi[k * D + a];
            c20 += (x - s0[1 + a]) * (x - s0[1 + a]);
            c21 += (x - s1[1 + a]) * (x - s1[1 + a]);
        }
        const double G0 = init ? 0.0 : n0 * exp(-c20 / (2 * s0[D + 1]));
        const double G1 = n1 * exp(-c21 / (2 * s1[D + 1]));
        const double dG[4] = {G1 - G0, 0.5 * dr * (s1[D + 2] * G1 - s0[D + 2] * G0),
                              Tvref > 0 ? ev1 * G1 - ev0 * G0 : 0.5 * dv * (s1[D + 3] * G1 - s0[D + 3] * G0),
                              (3 - D) * (s1[D + 1] * G1 - s0[D + 1] * G0)};
#pragma unroll
        for (int d = 0; d < ND; ++d) fv[d][e] = init ? (T)dG[d] : (T)((double)fv[d][e] + dG[d]);
      }
#pragma unroll
      for (int d = 0; d < ND; ++d) store_vw_nt<T, VW>(f + ((int64_t)c * ND + d) * nv + kb, fv[d]);
    }
    if (ch != 0) return;
    const double dI = init ? s1[D + 4] / (4 * kPi) : (s1[D + 4] - s0[D + 4]) / (4 * kPi);
    for (int64_t q0 = 0; q0 < no; q0 += kWave) {
        const int64_t q = q0 + lane;
        if (q >= no) break;
        const int64_t o = (int64_t)c * no + q;
        if (init)
            I[o] = (T)dI;
        else
            I[o] = (T)((double)I[o] + dI);
    }
}

// ------------------------------------------------------------------ launchers
static inline int64_t wave_blocks(int64_t n) { return (n + 3) / 4; }

// Cells per chunk-major group of the (cell, velocity chunk) kernels, measured (MI355X; 20k-triangle cavity,
// 1,024 velocities, 4 chunks; 214k-tetrahedron capsule, 1,728 velocities, 7 chunks, and 13,824 velocities,
// 54 chunks): the residual is fastest fully chunk-major in 2D and 3D (3D, 54 chunks: 60.3 ms against 89.4
// cell-major); the sweep fully chunk-major in 2D (5.82 against 5.53 TB/s) and in 3D with many chunks (54:
// 23.0 ms against 25.3 cell-major) but cell-major in 3D with few (7: 4.79 against 4.55 TB/s); the gradients
// chunk-major in 2D and cell-major in 3D (54 chunks: 35.3 ms against 40.2); the synchronisation with groups
// of 1,024 cells.
enum class CG { grad, residual, sweep, sync };
static int chunk_group(CG k, int D, int64_t ncell, int nchunk = 1)
{
    const int all = (int)ncell;
    switch (k) {
    case CG::residual: return all;
    case CG::sweep: return (D == 3 && nchunk < 16) ? 1 : all;
    case CG::grad: return D == 3 ? 1 : all;
    default: return (int)std::min<int64_t>(ncell, 1024);
    }
}

template <typename T, int D, int NFM>
void launch_grad(const T *f, T *gf, const MeshDev &m, int64_t nv, int so, const int *cells, int64_t ncl,
                 int compact, hipStream_t st)
{
    if (ncl <= 0) return;
    constexpr int VW = 16 / sizeof(T);
    if (nv % VW == 0) {
        const int nchunk = (int)((nv + kWave * VW - 1) / (kWave * VW));
        hipLaunchKernelGGL((k_grad_v<T, D, NFM, VW>), dim3(wave_blocks(ncl * nchunk)), dim3(256), 0, st, f, gf, m,
                           nv, nchunk, chunk_group(CG::grad, D, ncl), so, cells, ncl, compact);
    }
    else
        hipLaunchKernelGGL((k_grad<T, D, NFM>), dim3(wave_blocks(ncl)), dim3(256), 0, st, f, gf, m,
                           (D == 3) ? 3 : 4, nv, so, cells, ncl, compact);
}

// lanes per cell of the packed ordinate kernels: 2^ord_lsh(no) covers no / VW ordinates (at most 64)
static inline int ord_lsh(int64_t no, int vw)
{
    int l = 0;
    while (l < 6 && ((int64_t)vw << l) < no) ++l;
    return l;
}
static inline int64_t packed_blocks(int64_t ncells, int lsh) { return ((ncells << lsh) + 255) / 256; }

template <typename T, int D, int NFM>
void launch_grad_I(const T *I, T *gI, const MeshDev &m, int64_t no, int so, const int *cells, int64_t ncl,
                   hipStream_t st)
{
    if (ncl <= 0 || no <= 0) return;
    constexpr int VW = 16 / sizeof(T);
    if (no % VW == 0) {
        const int lsh = ord_lsh(no, VW);
        hipLaunchKernelGGL((k_grad_Iv<T, D, NFM, VW>), dim3(packed_blocks(ncl, lsh)), dim3(256), 0, st, I, gI, m,
                           no, lsh, so, cells, ncl);
    } else {
        hipLaunchKernelGGL((k_grad_I<T, D, NFM>), dim3(wave_blocks(ncl)), dim3(256), 0, st, I, gI, m, no, so,
                           cells, ncl);
    }
}

template <typename T>
__global__ void k_scale(T *__restrict__ f, const int64_t n, const double *__restrict__ num,
                        const double *__restrict__ den)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double sc = num[0] / den[0];
    f[i] = (T)((double)f[i] * sc);
}

template <typename T>
void launch_scale(T *f, int64_t n, const double *num, const double *den, hipStream_t st)
{
    hipLaunchKernelGGL(k_scale<T>, dim3((n + 255) / 256), dim3(256), 0, st, f, n, num, den);
}
template void launch_scale<float>(float *, int64_t, const double *, const double *, hipStream_t);
template void launch_scale<double>(double *, int64_t, const double *, const double *, hipStream_t);

// one colored Gauss-Seidel pass over the cells cl[0..ncl) of colour q (mode 0, 1 or 2 of k_sgs_v)
template <typename T, int D, int NFM, int VW>
static void sgs_pass_vw(int mode, const T *r, T *dl, T *f, const T *coef, const T *xiT, const MeshDev &m,
                        int64_t nv, T fac, T om, const int *cl, int ncl, int q, int upd, hipStream_t st)
{
    const int nchunk = (int)((nv + kWave * VW - 1) / (kWave * VW));
    const dim3 g((unsigned)(((int64_t)ncl * nchunk + 3) / 4)), blk(256);
    const int cg = chunk_group(CG::sweep, D, ncl);
    if (mode == 0)
        hipLaunchKernelGGL((k_sgs_v<T, D, NFM, VW, 0>), g, blk, 0, st, r, dl, f, coef, xiT, m, nv, nchunk, cg, fac, om,
                           cl, ncl, q, upd);
    else if (mode == 1)
        hipLaunchKernelGGL((k_sgs_v<T, D, NFM, VW, 1>), g, blk, 0, st, r, dl, f, coef, xiT, m, nv, nchunk, cg, fac, om,
                           cl, ncl, q, upd);
    else
        hipLaunchKernelGGL((k_sgs_v<T, D, NFM, VW, 2>), g, blk, 0, st, r, dl, f, coef, xiT, m, nv, nchunk, cg, fac, om,
                           cl, ncl, q, upd);
}

template <typename T, int D, int NFM>
static void sgs_pass(int mode, const T *r, T *dl, T *f, const T *coef, const T *xiT, const MeshDev &m, int64_t nv,
                     T fac, T om, const int *cl, int ncl, int q, int upd, hipStream_t st)
{
    constexpr int VW = 16 / sizeof(T);
    if (nv % VW == 0)
        sgs_pass_vw<T, D, NFM, VW>(mode, r, dl, f, coef, xiT, m, nv, fac, om, cl, ncl, q, upd, st);
    else
        sgs_pass_vw<T, D, NFM, 1>(mode, r, dl, f, coef, xiT, m, nv, fac, om, cl, ncl, q, upd, st);
}

template <typename T, int D, int NFM, int VW>
static void sgs_pass_I_vw(int mode, const T *r, T *dl, T *I, const T *coef, const T *om_, const MeshDev &m,
                          int64_t no, T fac, T om, T keff, const int *cl, int ncl, int q, int upd, hipStream_t st)
{
    const int lsh = ord_lsh(no, VW);
    const dim3 g((unsigned)packed_blocks(ncl, lsh)), blk(256);
    if (mode == 0)
        hipLaunchKernelGGL((k_sgs_Iv<T, D, NFM, VW, 0>), g, blk, 0, st, r, dl, I, coef, om_, m, no, lsh, fac, om, keff,
                           cl, ncl, q, upd);
    else if (mode == 1)
        hipLaunchKernelGGL((k_sgs_Iv<T, D, NFM, VW, 1>), g, blk, 0, st, r, dl, I, coef, om_, m, no, lsh, fac, om, keff,
                           cl, ncl, q, upd);
    else
        hipLaunchKernelGGL((k_sgs_Iv<T, D, NFM, VW, 2>), g, blk, 0, st, r, dl, I, coef, om_, m, no, lsh, fac, om, keff,
                           cl, ncl, q, upd);
}

template <typename T, int D, int NFM>
static void sgs_pass_I(int mode, const T *r, T *dl, T *I, const T *coef, const T *om_, const MeshDev &m, int64_t no,
                       T fac, T om, T keff, const int *cl, int ncl, int q, int upd, hipStream_t st)
{
    if (no <= 0) return;
    constexpr int VW = 16 / sizeof(T);
    if (no % VW == 0)
        sgs_pass_I_vw<T, D, NFM, VW>(mode, r, dl, I, coef, om_, m, no, fac, om, keff, cl, ncl, q, upd, st);
    else
        sgs_pass_I_vw<T, D, NFM, 1>(mode, r, dl, I, coef, om_, m, no, fac, om, keff, cl, ncl, q, upd, st);
}

template <typename T, int D, int NFM>
void launch_kinetic(KinBufs<T> &B, const MeshDev &m, const Phys &p, const KinOpts &o, int64_t nv, int64_t no,
                    hipStream_t st, Prof *pf)
{
    constexpr int ND = (D == 3) ? 3 : 4;
    const T fac = (T)(1.0 + 1.0 / o.cfl_v);
    const T om = (T)o.kin_omega;
    const T wt = (T)(1.0 - 1.0 / p.Z_r - 1.0 / p.Z_v), wr = (T)(1.0 / p.Z_r), wv = (T)(1.0 / p.Z_v);
    const dim3 grid(wave_blocks(m.nc)), blk(256);
    // algorithmic bytes of each launch: every array the kernel must touch, once
    const double es = sizeof(T), cv = (double)m.nc * nv * ND * es, co = (double)m.nc * no * es;
    Prof dummy;
    Prof &P = pf ? *pf : dummy;
    constexpr int VW = 16 / sizeof(T);
    // gradients recomputed inside the residual (vector kernels only); the stored pass otherwise.  Either way
    // the wall densities read gradient rows of the boundary cells: the compact rows of gfb, or gf itself.
    const bool fused = o.fused && (nv % VW == 0);
    const T *cons = o.conservative ? B.ccons : nullptr;  // discrete-conservative corrections, when enabled
    int ev = P.begin(0, fused ? (double)m.nbcells * nv * ND * es * (1 + D) : cv * (1 + D));
    if (fused) launch_grad<T, D, NFM>(B.f, B.gfb, m, nv, o.second_order, m.bcells, m.nbcells, 1, st);
    else launch_grad<T, D, NFM>(B.f, B.gf, m, nv, o.second_order, nullptr, m.nc, 0, st);
    P.end(ev);
    ev = P.begin(3, co * (1 + D));
    launch_grad_I<T, D, NFM>(B.I, B.gI, m, no, o.second_order, nullptr, m.nc, st);
    P.end(ev);
    ev = P.begin(5, 0.0);
    if (m.nbf > 0)
        hipLaunchKernelGGL((k_wall_density<T, D, NFM>), dim3(m.nbf), dim3(256), 0, st, B.f, fused ? B.gfb : B.gf,
                           fused ? m.bf_bidx : m.bf_cell, B.xi_d, B.w_d, B.rhow, m, nv);
    P.end(ev);
    const int ks = o.kin_sweeps;
    const double rbytes = (ks == 0 || o.sweep == 1) ? 2 * cv : 3 * cv;  // f read; r (and the first iterate) written
    ev = P.begin(1, fused ? rbytes : rbytes + cv * D);
    // vector kernels with one wave per (cell, chunk of kWave * VW velocities)
    const int nchunk = (int)((nv + kWave * VW - 1) / (kWave * VW));
    const dim3 chunk_grid((unsigned)((m.nc * nchunk + 3) / 4));
    const bool sgs = (o.sweep == 1);
    const bool direct = (!sgs && ks == 0);  // no sweeps: the residual writes f + omega r / d into f2
    if (fused) {
        // half-width vectors: the second ring of gradients needs the registers (occupancy 3 waves per SIMD)
        constexpr int VF = VW / 2;
        const int nchf = (int)((nv + kWave * VF - 1) / (kWave * VF));
        hipLaunchKernelGGL((k_gres_v<T, D, NFM, VF>), dim3((unsigned)((m.nc * nchf + 3) / 4)), blk, 0, st, B.f,
                           B.coef, cons, B.xiT, B.rhow, B.r, sgs ? nullptr : B.dl0, direct ? B.f2 : nullptr, m, nv, nchf,
                           chunk_group(CG::residual, D, m.nc), o.second_order, fac, om, wt, wr, wv, (T)p.d_r,
                           (T)p.d_v);
    }
    else if (nv % VW == 0)
        hipLaunchKernelGGL((k_residual_v<T, D, NFM, VW>), chunk_grid, blk, 0, st, B.f, B.gf, B.coef, cons, B.xiT,
                           B.rhow,
                           B.r, sgs ? nullptr : B.dl0, direct ? B.f2 : nullptr, m, nv, nchunk,
                           chunk_group(CG::residual, D, m.nc), fac, om, wt, wr, wv, (T)p.d_r, (T)p.d_v);
    else
        hipLaunchKernelGGL((k_residual<T, D, NFM>), grid, blk, 0, st, B.f, B.gf, B.coef, cons, B.xi, B.rhow, B.r,
                           sgs ? nullptr : B.dl0, direct ? B.f2 : nullptr, m, nv, fac, om, wt, wr, wv, (T)p.d_r,
                           (T)p.d_v);
    P.end(ev);
    ev = P.begin(3, ks == 0 ? co * (2 + D) : co * (3 + D));
    const bool ovec = (no % VW == 0);
    const int olsh = ord_lsh(no, VW);
    const dim3 ogrid((unsigned)packed_blocks(m.nc, olsh));
    if (ovec)
        hipLaunchKernelGGL((k_residual_Iv<T, D, NFM, VW>), ogrid, blk, 0, st, B.I, B.gI, B.coef, B.om, B.rI,
                           sgs ? nullptr : B.dI0, direct ? B.I2 : nullptr, m, no, olsh, fac, om, (T)p.keff,
                           (T)p.sigma_R);
    else
        hipLaunchKernelGGL((k_residual_I<T, D, NFM>), grid, blk, 0, st, B.I, B.gI, B.coef, B.om, B.rI,
                           sgs ? nullptr : B.dI0, direct ? B.I2 : nullptr, m, no, fac, om, (T)p.keff, (T)p.sigma_R);
    P.end(ev);
    if (o.sweep == 1) {
        // colored symmetric Gauss-Seidel: nsw symmetric sweeps, each a forward pass over the colours in
        // ascending order and a backward pass in descending order; one sweep runs in place in r
        const int nsw = ks > 0 ? ks : 1;
        T *dbuf = (nsw == 1) ? B.r : B.dl0;
        T *dIbuf = (nsw == 1) ? B.rI : B.dI0;
        for (int sw = 0; sw < nsw; ++sw)
            for (int pass = 0; pass < 2; ++pass)
                for (int qq = 0; qq < o.ncolor; ++qq) {
                    const int q = (pass == 0) ? qq : o.ncolor - 1 - qq;
                    const int mode = (sw == 0) ? pass : 2;
                    const int last = (sw == nsw - 1 && pass == 1) ? 1 : 0;
                    const int ncl = (int)(o.col_ptr[q + 1] - o.col_ptr[q]);
                    if (ncl <= 0) continue;
                    const int *cl = m.col_cells + o.col_ptr[q];
                    const double own = (double)ncl * nv * ND * es;
                    ev = P.begin(2, own * (last ? 4 : 2));
                    sgs_pass<T, D, NFM>(mode, B.r, dbuf, B.f, B.coef, B.xiT, m, nv, fac, om, cl, ncl, q, last, st);
                    P.end(ev);
                    ev = P.begin(3, (double)ncl * no * es * (last ? 4 : 2));
                    sgs_pass_I<T, D, NFM>(mode, B.rI, dIbuf, B.I, B.coef, B.om, m, no, fac, om, (T)p.keff, cl, ncl, q,
                                          last, st);
                    P.end(ev);
                }
        return;
    }
    // Jacobi sweeps; the last one writes f + omega Delta in place (each element is read and written by the
    // same lane, and no sweep reads f of another cell)
    T *din = B.dl0, *dout = B.dl1, *dIin = B.dI0, *dIout = B.dI1;
    for (int s = 0; s < ks; ++s) {
        const bool last = (s == ks - 1);
        ev = P.begin(2, last ? 4 * cv : 3 * cv);
        if (nv % VW == 0)
            hipLaunchKernelGGL((k_sweep_v<T, D, NFM, VW>), chunk_grid, blk, 0, st, B.r, din, dout, B.f,
                               last ? B.f : nullptr, B.coef, B.xiT, m, nv, nchunk,
                               chunk_group(CG::sweep, D, m.nc, nchunk), fac, om);
        else
            hipLaunchKernelGGL((k_sweep<T, D, NFM>), grid, blk, 0, st, B.r, din, dout, B.f, last ? B.f : nullptr,
                               B.coef, B.xi, m, nv, fac, om);
        P.end(ev);
        ev = P.begin(3, last ? 4 * co : 3 * co);
        if (ovec)
            hipLaunchKernelGGL((k_sweep_Iv<T, D, NFM, VW>), ogrid, blk, 0, st, B.rI, dIin, dIout, B.I,
                               last ? B.I : nullptr, B.coef, B.om, m, no, olsh, fac, om, (T)p.keff);
        else
            hipLaunchKernelGGL((k_sweep_I<T, D, NFM>), grid, blk, 0, st, B.rI, dIin, dIout, B.I,
                               last ? B.I : nullptr, B.coef, B.om, m, no, fac, om, (T)p.keff);
        P.end(ev);
        std::swap(din, dout);
        std::swap(dIin, dIout);
    }
    if (ks == 0) {
        std::swap(B.f, B.f2);
        std::swap(B.I, B.I2);
    }
}

template <typename T, int D>
void launch_moments(const KinBufs<T> &B, const double *uref, double *mom, int64_t nc, int64_t nv, int64_t no,
                    const Phys &p, hipStream_t st)
{
    constexpr int VW = 16 / sizeof(T);
    const int64_t mom_blocks = (nc + 256 / kMomLanes - 1) / (256 / kMomLanes);
    if (nv % VW == 0)
        hipLaunchKernelGGL((k_moments<T, D, VW>), dim3(mom_blocks), dim3(256), 0, st, B.f, B.I, B.xi_d, B.w_d, B.om_d,
                           B.wo_d, uref, mom, nc, nv, no, p.d_r, p.d_v, p.Tvref);
    else
        hipLaunchKernelGGL((k_moments<T, D, 1>), dim3(mom_blocks), dim3(256), 0, st, B.f, B.I, B.xi_d, B.w_d, B.om_d,
                           B.wo_d, uref, mom, nc, nv, no, p.d_r, p.d_v, p.Tvref);
}

template <typename T, int D>
void launch_prologue(const double *mom, T *coef, const double *h, int64_t nc, const Phys &p, double cfl,
                     hipStream_t st)
{
    hipLaunchKernelGGL((k_prologue<T, D>), dim3((nc + 255) / 256), dim3(256), 0, st, mom, coef, h, nc, p, cfl);
}

template <typename T, int D, int NFM>
void launch_boundary_state(KinBufs<T> &B, const MeshDev &m, const Phys &p, int so, int64_t nv, int64_t no,
                           hipStream_t st)
{
    if (m.nbf <= 0) return;
    // gradient rows of the boundary cells only, compact (row i for the i-th boundary cell)
    launch_grad<T, D, NFM>(B.f, B.gfb, m, nv, so, m.bcells, m.nbcells, 1, st);
    launch_grad_I<T, D, NFM>(B.I, B.gI, m, no, so, m.bcells, m.nbcells, st);
    hipLaunchKernelGGL((k_wall_density<T, D, NFM>), dim3(m.nbf), dim3(256), 0, st, B.f, B.gfb, m.bf_bidx, B.xi_d,
                       B.w_d, B.rhow, m, nv);
    hipLaunchKernelGGL((k_boundary_flux<T, D>), dim3(m.nbf), dim3(256), 0, st, B.f, B.gfb, m.bf_bidx, B.I, B.gI,
                       B.xi_d, B.w_d,
                       B.om_d, B.wo_d, B.rhow, B.bflux, B.bsurf, m, nv, no, p.d_r, p.d_v, p.sigma_R);
}

template <typename T, int D>
void launch_sync(KinBufs<T> &B, const double *sp, int64_t nc, int64_t nv, int64_t no, const Phys &p, int init,
                 hipStream_t st)
{
    constexpr int VW = 16 / sizeof(T);
    if (nv % VW == 0) {
        const int nchunk = (int)((nv + kWave * VW - 1) / (kWave * VW));
        hipLaunchKernelGGL((k_sync<T, D, VW>), dim3(wave_blocks(nc * nchunk)), dim3(256), 0, st, B.f, B.I, sp,
                           B.xi_d, nc, nv, nchunk, chunk_group(CG::sync, D, nc), no, p.d_r, p.d_v, p.Tvref, init);
    } else {
        const int nchunk = (int)((nv + kWave - 1) / kWave);
        hipLaunchKernelGGL((k_sync<T, D, 1>), dim3(wave_blocks(nc * nchunk)), dim3(256), 0, st, B.f, B.I, sp,
                           B.xi_d, nc, nv, nchunk, chunk_group(CG::sync, D, nc), no, p.d_r, p.d_v, p.Tvref, init);
    }
}

#define GSIS_INST_D(T, D, NFM)                                                                                    \
    template void launch_kinetic<T, D, NFM>(KinBufs<T> &, const MeshDev &, const Phys &, const KinOpts &, int64_t, \
                                            int64_t, hipStream_t, Prof *);                                        \
    template void launch_boundary_state<T, D, NFM>(KinBufs<T> &, const MeshDev &, const Phys &, int, int64_t,     \
                                                   int64_t, hipStream_t);
#define GSIS_INST_T(T, D)                                                                                          \
    template void launch_moments<T, D>(const KinBufs<T> &, const double *, double *, int64_t, int64_t, int64_t,   \
                                       const Phys &, hipStream_t);                                                 \
    template void launch_prologue<T, D>(const double *, T *, const double *, int64_t, const Phys &, double,       \
                                        hipStream_t);                                                              \
    template void launch_cons_sums<T, D>(const double *, const T *, const T *, const double *, T *, int64_t,      \
                                         int64_t, const Phys &, hipStream_t);                                     \
    template void launch_sync<T, D>(KinBufs<T> &, const double *, int64_t, int64_t, int64_t, const Phys &, int,   \
                                    hipStream_t);

GSIS_INST_D(float, 1, 2)
GSIS_INST_D(double, 1, 2)
GSIS_INST_D(float, 2, 3)
GSIS_INST_D(double, 2, 3)
GSIS_INST_D(float, 2, 4)
GSIS_INST_D(double, 2, 4)
GSIS_INST_D(float, 3, 4)
GSIS_INST_D(double, 3, 4)
GSIS_INST_D(float, 3, 6)
GSIS_INST_D(double, 3, 6)
GSIS_INST_T(float, 1)
GSIS_INST_T(double, 1)
GSIS_INST_T(float, 2)
GSIS_INST_T(double, 2)
GSIS_INST_T(float, 3)
GSIS_INST_T(double, 3)

}  // namespace gsis
