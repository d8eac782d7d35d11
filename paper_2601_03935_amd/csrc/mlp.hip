// Warm-start network on gfx950 (declarations and documentation in include/gsis_warmstart.h): a 4-layer
// perceptron with BF16 weights and FP32 accumulation; forward, mean-squared-error backward and Adam, all in
// HIP kernels.  With BF16 weights every product runs on the matrix cores (both operands rounded to BF16 in
// LDS, FP32 accumulation); with FP32 weights on the vector ALUs (64 x 64 outputs per 256-thread workgroup,
// 4 x 4 per thread).  k is summed in a fixed order; column sums and the loss use two-pass fixed-order
// reductions, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gsis.h"
#include "../../include/gsis_warmstart.h"
#include "gsis_kernels.h"

namespace {

constexpr int kLayers = 4;
constexpr int TBM = 64, TBN = 64, TBK = 16;

__host__ __device__ inline uint16_t f32_to_bf16(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float ld(const float *p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ld(const uint16_t *p, int64_t i)
{
    return __builtin_bit_cast(float, (uint32_t)p[i] << 16);
}

enum { EPI_BIAS_TANH = 0, EPI_BIAS = 1, EPI_DTANH = 2, EPI_STORE = 3 };

// C[m][n] = epilogue(sum_k A(m,k) B(k,n)) with A(m,k) = TA ? A[k lda + m] : A[m lda + k] and
// B(k,n) = TB ? B[n ldb + k] : B[k ldb + n].
template <bool TA, bool TB, typename BT, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const int M, const int N, const int K, const float *__restrict__ A,
                                              const int lda, const BT *__restrict__ B, const int ldb,
                                              float *__restrict__ C, const int ldc, const float *__restrict__ bias,
                                              const float *__restrict__ aux)
{
    __shared__ float As[TBK][TBM + 4];
    __shared__ float Bs[TBK][TBN + 4];
    const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
    const int m0 = blockIdx.y * TBM, n0 = blockIdx.x * TBN;
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
    for (int k0 = 0; k0 < K; k0 += TBK) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = t + 256 * e;
            int mm, kk;
            if (TA) {
                mm = idx % TBM;
                kk = idx / TBM;
            } else {
                kk = idx % TBK;
                mm = idx / TBK;
            }
            const int m = m0 + mm, k = k0 + kk;
            float v = 0.f;
            if (m < M && k < K) v = TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
            As[kk][mm] = v;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = t + 256 * e;
            int nn, kk;
            if (TB) {
                kk = idx % TBK;
                nn = idx / TBK;
            } else {
                nn = idx % TBN;
                kk = idx / TBN;
            }
            const int n = n0 + nn, k = k0 + kk;
            float v = 0.f;
            if (n < N && k < K) v = TB ? ld(B, (int64_t)n * ldb + k) : ld(B, (int64_t)k * ldb + n);
            Bs[kk][nn] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TBK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + ty * 4 + i;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + tx * 4 + j;
            if (n >= N) continue;
            const int64_t o = (int64_t)m * ldc + n;
            float v = acc[i][j];
            if (EPI == EPI_BIAS_TANH) {
                v = tanhf(v + bias[n]);
            } else if (EPI == EPI_BIAS) {
                v = v + bias[n];
            } else if (EPI == EPI_DTANH) {
                const float a = aux[o];
                v = v * (1.f - a * a);
            }
            C[o] = v;
        }
    }
}

// BF16 matrix-core form of the same product (used when the weights are BF16): both operands are rounded to
// BF16 (round to nearest even) while they are staged in LDS, products accumulate in FP32 with
// v_mfma_f32_32x32x8bf16.  Workgroup: 4 waves, 64 x 64 outputs, each wave a 32 x 32 block; k advances by
// 32 per LDS stage (four 8-deep MFMA steps), so every output sums its k terms in a fixed order.
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
constexpr int MBK = 32, MPAD = 8;

__device__ __forceinline__ float ldf(const float *p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldf(const uint16_t *p, int64_t i)
{
    return __builtin_bit_cast(float, (uint32_t)p[i] << 16);
}

template <bool TA, bool TB, typename BT, int EPI>
__global__ __launch_bounds__(256) void k_gemm_mfma(const int M, const int N, const int K,
                                                   const float *__restrict__ A, const int lda,
                                                   const BT *__restrict__ B, const int ldb, float *__restrict__ C,
                                                   const int ldc, const float *__restrict__ bias,
                                                   const float *__restrict__ aux)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[TBM][MBK + MPAD];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TBN][MBK + MPAD];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * TBM, n0 = blockIdx.x * TBN;
    f32x16_t acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
    for (int k0 = 0; k0 < K; k0 += MBK) {
        // stage A (64 x 32) and B (32 x 64): 8 consecutive elements of the contiguous index per thread
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int mm, kk;
            if (TA) {
                kk = t >> 3;
                mm = ((t & 7) << 3) + e;
            } else {
                mm = t >> 2;
                kk = ((t & 3) << 3) + e;
            }
            const int m = m0 + mm, k = k0 + kk;
            float v = 0.f;
            if (m < M && k < K) v = TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
            As[mm][kk] = f32_to_bf16(v);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int nn, kk;
            if (TB) {
                nn = t >> 2;
                kk = ((t & 3) << 3) + e;
            } else {
                kk = t >> 3;
                nn = ((t & 7) << 3) + e;
            }
            const int n = n0 + nn, k = k0 + kk;
            float v = 0.f;
            if (n < N && k < K) v = TB ? ldf(B, (int64_t)n * ldb + k) : ldf(B, (int64_t)k * ldb + n);
            Bs[nn][kk] = f32_to_bf16(v);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < MBK; kk += 8) {
            const int kc = kk + 4 * (lane >> 5);
            const bf16x4_t a = *(const bf16x4_t *)&As[wm * 32 + (lane & 31)][kc];
            const bf16x4_t b = *(const bf16x4_t *)&Bs[wn * 32 + (lane & 31)][kc];
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    const int n = n0 + wn * 32 + (lane & 31);
    if (n >= N) return;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int m = m0 + wm * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (m >= M) continue;
        const int64_t o = (int64_t)m * ldc + n;
        float x = acc[v];
        if (EPI == EPI_BIAS_TANH) {
            x = tanhf(x + bias[n]);
        } else if (EPI == EPI_BIAS) {
            x = x + bias[n];
        } else if (EPI == EPI_DTANH) {
            const float a = aux[o];
            x = x * (1.f - a * a);
        }
        C[o] = x;
    }
}

// column sums of X [M][N] in two fixed-order passes: partial sums over 256-row chunks, then over chunks
constexpr int kColRows = 256;
__global__ void k_colsum_part(const int M, const int N, const float *__restrict__ X, float *__restrict__ part)
{
    const int n = blockIdx.y * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int r0 = blockIdx.x * kColRows, r1 = min(M, r0 + kColRows);
    float s = 0.f;
    for (int r = r0; r < r1; ++r) s += X[(int64_t)r * N + n];
    part[(int64_t)blockIdx.x * N + n] = s;
}

__global__ void k_colsum_final(const int nchunk, const int N, const float *__restrict__ part, float *__restrict__ out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * N + n];
    out[n] = s;
}

// dY = 2 (y - t) / (n n_out); per-block sums of (y - t)^2 in FP64
__global__ __launch_bounds__(256) void k_mse(const int64_t cnt, const float *__restrict__ y,
                                             const float *__restrict__ t, const float scale, float *__restrict__ dy,
                                             double *__restrict__ part)
{
    __shared__ double sh[256];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double e2 = 0;
    if (i < cnt) {
        const float d = y[i] - t[i];
        dy[i] = scale * d;
        e2 = (double)d * (double)d;
    }
    sh[threadIdx.x] = e2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_sum_final(const int nb, const double *__restrict__ part, const double scale,
                                                   double *__restrict__ out)
{
    __shared__ double sh[256];
    double s = 0;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[b];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] * scale;
}

__global__ void k_adam(const int64_t np, float *__restrict__ P, const float *__restrict__ G, float *__restrict__ Mm,
                       float *__restrict__ Vv, uint16_t *__restrict__ Ph, const float lr, const float b1,
                       const float b2, const float eps, const float bc1, const float bc2)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float g = G[i];
    const float m = b1 * Mm[i] + (1.f - b1) * g;
    const float v = b2 * Vv[i] + (1.f - b2) * g * g;
    Mm[i] = m;
    Vv[i] = v;
    const float p = P[i] - lr * (m / bc1) / (sqrtf(v / bc2) + eps);
    P[i] = p;
    Ph[i] = f32_to_bf16(p);
}

__global__ void k_to_bf16(const int64_t np, const float *__restrict__ P, uint16_t *__restrict__ Ph)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < np) Ph[i] = f32_to_bf16(P[i]);
}

__global__ void k_gather_rows(const int64_t nb, const int *__restrict__ idx, const int w,
                              const float *__restrict__ src, float *__restrict__ dst)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nb * w) return;
    const int64_t r = i / w, c = i % w;
    dst[i] = src[(int64_t)idx[r] * w + c];
}

uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t &s) { return (double)(splitmix64(s) >> 11) * 0x1.0p-53; }

}  // namespace

struct gsis_mlp_s {
    int device = 0;
    hipStream_t st = nullptr;
    int n_in = 0, width = 0, n_out = 0;
    bool bf16 = true;
    int in_[kLayers] = {0}, out_[kLayers] = {0};
    int64_t offW[kLayers] = {0}, offb[kLayers] = {0}, np = 0;
    float *P = nullptr, *G = nullptr, *Mm = nullptr, *Vv = nullptr;
    uint16_t *Ph = nullptr;
    int64_t cap = 0;
    float *X = nullptr, *T = nullptr, *Y = nullptr, *dY = nullptr, *A[3] = {nullptr, nullptr, nullptr};
    float *dZ[2] = {nullptr, nullptr}, *cpart = nullptr;
    double *lpart = nullptr, *loss = nullptr;
    int64_t adam_t = 0;
    float *scratch = nullptr;  // this device's copy of the file-scope scratch array (hipGetSymbolAddress)
    std::string err;
};

// Hidden activations of gsis_mlp_forward_noalloc: a file-scope device array, one copy per GPU, held until the
// process ends.  In host code the symbol is only a stand-in; kernels get the address hipGetSymbolAddress
// returns with the device current (kept per device below).
constexpr int64_t kScratchFloats = (int64_t)1 << 21;  // 8 MiB
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch[kMaxDevices] = {};

// address of the scratch array on `device`, which must be the current device; nullptr if the lookup fails
float *scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch[device] = (float *)p;
    }
    return g_scratch[device];
}

int32_t fail(gsis_mlp_t *m, int32_t code, const std::string &msg)
{
    m->err = msg;
    return code;
}

#define MCHECK(m, expr)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail(m, GSIS_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
bool dalloc(T *&p, int64_t n)
{
    p = nullptr;
    return hipMalloc((void **)&p, std::max<int64_t>(n, 1) * sizeof(T)) == hipSuccess;
}

template <typename T>
void dfree(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_batch(gsis_mlp_t *m)
{
    dfree(m->X);
    dfree(m->T);
    dfree(m->Y);
    dfree(m->dY);
    for (auto &a : m->A) dfree(a);
    for (auto &d : m->dZ) dfree(d);
    dfree(m->cpart);
    dfree(m->lpart);
    m->cap = 0;
}

bool ensure_batch(gsis_mlp_t *m, int64_t n)
{
    if (n <= m->cap) return true;
    free_batch(m);
    const int64_t w = m->width;
    bool ok = dalloc(m->X, n * m->n_in) && dalloc(m->T, n * m->n_out) && dalloc(m->Y, n * m->n_out) &&
              dalloc(m->dY, n * m->n_out) && dalloc(m->A[0], n * w) && dalloc(m->A[1], n * w) &&
              dalloc(m->A[2], n * w) && dalloc(m->dZ[0], n * w) && dalloc(m->dZ[1], n * w) &&
              dalloc(m->cpart, ((n + kColRows - 1) / kColRows) * std::max<int64_t>({w, m->n_in, m->n_out})) &&
              dalloc(m->lpart, (n * m->n_out + 255) / 256);
    if (!ok) {
        free_batch(m);
        return false;
    }
    m->cap = n;
    return true;
}

// products: BF16 matrix cores when the network runs with BF16 weights, FP32 vector ALUs otherwise
template <bool TA, bool TB, typename BT, int EPI>
void gemm(gsis_mlp_t *m, int M, int N, int K, const float *A, int lda, const BT *B, int ldb, float *C, int ldc,
          const float *bias, const float *aux)
{
    const dim3 grid((N + TBN - 1) / TBN, (M + TBM - 1) / TBM);
    if (m->bf16)
        hipLaunchKernelGGL((k_gemm_mfma<TA, TB, BT, EPI>), grid, dim3(256), 0, m->st, M, N, K, A, lda, B, ldb, C, ldc,
                           bias, aux);
    else
        hipLaunchKernelGGL((k_gemm<TA, TB, BT, EPI>), grid, dim3(256), 0, m->st, M, N, K, A, lda, B, ldb, C, ldc,
                           bias, aux);
}

// weights of layer l as the product kernels read them
template <typename BT>
const BT *wptr(gsis_mlp_t *m, int l);
template <>
const float *wptr<float>(gsis_mlp_t *m, int l)
{
    return m->P + m->offW[l];
}
template <>
const uint16_t *wptr<uint16_t>(gsis_mlp_t *m, int l)
{
    return m->Ph + m->offW[l];
}

// n rows of X [n][n_in] through the four layers into Y [n][n_out], hidden activations in H0, H1, H2 ([n][width]
// each; H2 may be H0, which layer 2 does not read)
template <typename BT>
void forward_T(gsis_mlp_t *m, int n, const float *X, float *H0, float *H1, float *H2, float *Y)
{
    const int w = m->width;
    gemm<false, true, BT, EPI_BIAS_TANH>(m, n, w, m->n_in, X, m->n_in, wptr<BT>(m, 0), m->n_in, H0, w,
                                         m->P + m->offb[0], nullptr);
    gemm<false, true, BT, EPI_BIAS_TANH>(m, n, w, w, H0, w, wptr<BT>(m, 1), w, H1, w, m->P + m->offb[1], nullptr);
    gemm<false, true, BT, EPI_BIAS_TANH>(m, n, w, w, H1, w, wptr<BT>(m, 2), w, H2, w, m->P + m->offb[2], nullptr);
    gemm<false, true, BT, EPI_BIAS>(m, n, m->n_out, w, H2, w, wptr<BT>(m, 3), w, Y, m->n_out, m->P + m->offb[3],
                                    nullptr);
}

void forward_rows(gsis_mlp_t *m, int n, const float *X, float *H0, float *H1, float *H2, float *Y)
{
    if (m->bf16) forward_T<uint16_t>(m, n, X, H0, H1, H2, Y);
    else forward_T<float>(m, n, X, H0, H1, H2, Y);
}

// the handle's batch buffers (every activation kept for the backward pass)
void forward(gsis_mlp_t *m, int n) { forward_rows(m, n, m->X, m->A[0], m->A[1], m->A[2], m->Y); }

void colsum(gsis_mlp_t *m, int M, int N, const float *X, float *out)
{
    const int nchunk = (M + kColRows - 1) / kColRows;
    hipLaunchKernelGGL(k_colsum_part, dim3(nchunk, (N + 255) / 256), dim3(256), 0, m->st, M, N, X, m->cpart);
    hipLaunchKernelGGL(k_colsum_final, dim3((N + 255) / 256), dim3(256), 0, m->st, nchunk, N, m->cpart, out);
}

// loss into m->loss (device) and gradient into m->G, for the n rows in X, T
template <typename BT>
void backward_T(gsis_mlp_t *m, int n)
{
    const int w = m->width, no = m->n_out;
    const int64_t cnt = (int64_t)n * no;
    const int nb = (int)((cnt + 255) / 256);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, m->st, cnt, m->Y, m->T, (float)(2.0 / (double)cnt), m->dY,
                       m->lpart);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, m->st, nb, m->lpart, 1.0 / (double)cnt, m->loss);
    float *G = m->G;
    // layer 4
    gemm<true, false, float, EPI_STORE>(m, no, w, n, m->dY, no, m->A[2], w, G + m->offW[3], w, nullptr, nullptr);
    colsum(m, n, no, m->dY, G + m->offb[3]);
    gemm<false, false, BT, EPI_DTANH>(m, n, w, no, m->dY, no, wptr<BT>(m, 3), w, m->dZ[0], w, nullptr, m->A[2]);
    // layer 3
    gemm<true, false, float, EPI_STORE>(m, w, w, n, m->dZ[0], w, m->A[1], w, G + m->offW[2], w, nullptr, nullptr);
    colsum(m, n, w, m->dZ[0], G + m->offb[2]);
    gemm<false, false, BT, EPI_DTANH>(m, n, w, w, m->dZ[0], w, wptr<BT>(m, 2), w, m->dZ[1], w, nullptr, m->A[1]);
    // layer 2
    gemm<true, false, float, EPI_STORE>(m, w, w, n, m->dZ[1], w, m->A[0], w, G + m->offW[1], w, nullptr, nullptr);
    colsum(m, n, w, m->dZ[1], G + m->offb[1]);
    gemm<false, false, BT, EPI_DTANH>(m, n, w, w, m->dZ[1], w, wptr<BT>(m, 1), w, m->dZ[0], w, nullptr, m->A[0]);
    // layer 1
    gemm<true, false, float, EPI_STORE>(m, w, m->n_in, n, m->dZ[0], w, m->X, m->n_in, G + m->offW[0], m->n_in,
                                        nullptr, nullptr);
    colsum(m, n, w, m->dZ[0], G + m->offb[0]);
}

void backward(gsis_mlp_t *m, int n)
{
    if (m->bf16) backward_T<uint16_t>(m, n);
    else backward_T<float>(m, n);
}

void adam(gsis_mlp_t *m, const gsis_mlp_train_opts *o)
{
    m->adam_t += 1;
    const double bc1 = 1.0 - std::pow(o->beta1, (double)m->adam_t), bc2 = 1.0 - std::pow(o->beta2, (double)m->adam_t);
    hipLaunchKernelGGL(k_adam, dim3((m->np + 255) / 256), dim3(256), 0, m->st, m->np, m->P, m->G, m->Mm, m->Vv, m->Ph,
                       (float)o->lr, (float)o->beta1, (float)o->beta2, (float)o->eps, (float)bc1, (float)bc2);
}

int32_t check_rows(gsis_mlp_t *m, int64_t n, const void *x)
{
    if (!x || n <= 0) return fail(m, GSIS_E_ARG, "row count must be positive and arrays non-null");
    if (n > (int64_t)INT32_MAX / 1024) return fail(m, GSIS_E_ARG, "too many rows in one call");
    return GSIS_OK;
}

int32_t upload_rows(gsis_mlp_t *m, int64_t n, const float *x, const float *t)
{
    if (!ensure_batch(m, n)) return fail(m, GSIS_E_OOM, "batch buffers: device allocation failed");
    MCHECK(m, hipMemcpyAsync(m->X, x, n * m->n_in * sizeof(float), hipMemcpyHostToDevice, m->st));
    if (t) MCHECK(m, hipMemcpyAsync(m->T, t, n * m->n_out * sizeof(float), hipMemcpyHostToDevice, m->st));
    return GSIS_OK;
}

// minibatch Adam over n device rows Xall [n][n_in], Tall [n][n_out] (host-shuffled order per epoch)
int32_t train_device(gsis_mlp_t *m, int64_t n, const float *Xall, const float *Tall, const gsis_mlp_train_opts *o,
                     double *final_loss)
{
    const int64_t bs = std::min<int64_t>(o->batch, n);
    const int64_t nbat = (n + bs - 1) / bs;
    if (!ensure_batch(m, bs)) return fail(m, GSIS_E_OOM, "training: device allocation failed");
    int *idx = nullptr;
    double *lossv = nullptr;
    struct Guard {
        int *&c;
        double *&d;
        ~Guard()
        {
            dfree(c);
            dfree(d);
        }
    } guard{idx, lossv};
    if (!(dalloc(idx, n) && dalloc(lossv, nbat))) return fail(m, GSIS_E_OOM, "training: device allocation failed");
    std::vector<int> perm(n);
    uint64_t s = o->seed;
    for (int ep = 0; ep < o->epochs; ++ep) {
        for (int64_t i = 0; i < n; ++i) perm[i] = (int)i;
        for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[(int64_t)(uniform01(s) * (double)(i + 1))]);
        MCHECK(m, hipMemcpyAsync(idx, perm.data(), n * sizeof(int), hipMemcpyHostToDevice, m->st));
        for (int64_t b = 0; b < nbat; ++b) {
            const int64_t r0 = b * bs, nr = std::min(bs, n - r0);
            hipLaunchKernelGGL(k_gather_rows, dim3((nr * m->n_in + 255) / 256), dim3(256), 0, m->st, nr, idx + r0,
                               m->n_in, Xall, m->X);
            hipLaunchKernelGGL(k_gather_rows, dim3((nr * m->n_out + 255) / 256), dim3(256), 0, m->st, nr, idx + r0,
                               m->n_out, Tall, m->T);
            forward(m, (int)nr);
            backward(m, (int)nr);
            adam(m, o);
            MCHECK(m, hipMemcpyAsync(lossv + b, m->loss, sizeof(double), hipMemcpyDeviceToDevice, m->st));
        }
        // the permutation buffer is rewritten next epoch: wait for this epoch's gathers
        MCHECK(m, hipStreamSynchronize(m->st));
    }
    if (final_loss) {
        std::vector<double> lv(nbat);
        MCHECK(m, hipMemcpy(lv.data(), lossv, nbat * sizeof(double), hipMemcpyDeviceToHost));
        double sum = 0;
        for (double v : lv) sum += v;
        *final_loss = o->epochs > 0 ? sum / (double)nbat : 0.0;
    }
    return GSIS_OK;
}

__global__ void k_standardize(const double *__restrict__ x, const double *__restrict__ mean,
                              const double *__restrict__ scale, float *__restrict__ out, const int64_t n, const int k)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * k) return;
    const int j = (int)(i % k);
    out[i] = (float)((x[i] - mean[j]) / scale[j]);
}

__global__ void k_destandardize(const float *__restrict__ y, const double *__restrict__ mean,
                                const double *__restrict__ scale, double *__restrict__ out, const int64_t n, const int k)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * k) return;
    const int j = (int)(i % k);
    out[i] = (double)y[i] * scale[j] + mean[j];
}

// the four standardisation vectors of a norm on the device (x_mean, x_scale, y_mean, y_scale, 64 each)
int32_t upload_norm(gsis_mlp_t *m, const gsis_ws_norm *norm, double *&d)
{
    if (!norm || norm->n_in != m->n_in || norm->n_out != m->n_out)
        return fail(m, GSIS_E_ARG, "standardisation dimensions differ from the network's");
    for (int j = 0; j < m->n_in; ++j)
        if (!(norm->x_scale[j] > 0)) return fail(m, GSIS_E_ARG, "non-positive input scale");
    for (int j = 0; j < m->n_out; ++j)
        if (!(norm->y_scale[j] > 0)) return fail(m, GSIS_E_ARG, "non-positive output scale");
    if (!dalloc(d, 4 * 64)) return fail(m, GSIS_E_OOM, "device allocation failed");
    MCHECK(m, hipMemcpyAsync(d, norm->x_mean, 64 * sizeof(double), hipMemcpyHostToDevice, m->st));
    MCHECK(m, hipMemcpyAsync(d + 64, norm->x_scale, 64 * sizeof(double), hipMemcpyHostToDevice, m->st));
    MCHECK(m, hipMemcpyAsync(d + 128, norm->y_mean, 64 * sizeof(double), hipMemcpyHostToDevice, m->st));
    MCHECK(m, hipMemcpyAsync(d + 192, norm->y_scale, 64 * sizeof(double), hipMemcpyHostToDevice, m->st));
    return GSIS_OK;
}

}  // namespace

namespace gsis {

float *mlp_input_rows(gsis_mlp_t *m, int64_t n) { return ensure_batch(m, n) ? m->X : nullptr; }

const float *mlp_forward_rows(gsis_mlp_t *m, int64_t n, hipStream_t st)
{
    hipStream_t keep = m->st;
    m->st = st;
    forward(m, (int)n);
    m->st = keep;
    return m->Y;
}

void mlp_dims(const gsis_mlp_t *m, int *n_in, int *n_out)
{
    *n_in = m->n_in;
    *n_out = m->n_out;
}

void launch_standardize(const double *x, const double *mean, const double *scale, float *out, int64_t n, int k,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_standardize, dim3((unsigned)((n * k + 255) / 256)), dim3(256), 0, st, x, mean, scale, out, n, k);
}

}  // namespace gsis

extern "C" {

int32_t gsis_mlp_create(int32_t device, int32_t n_in, int32_t width, int32_t n_out, int32_t bf16_weights,
                        uint64_t seed, gsis_mlp_t **out)
{
    if (!out) return GSIS_E_ARG;
    *out = nullptr;
    if (n_in < 1 || n_in > 64 || n_out < 1 || n_out > 64 || width < 1 || width > 1024) return GSIS_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GSIS_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return GSIS_E_DEVICE;
    auto *m = new gsis_mlp_t();
    m->device = device;
    m->n_in = n_in;
    m->width = width;
    m->n_out = n_out;
    m->bf16 = bf16_weights != 0;
    const int ins[kLayers] = {n_in, width, width, width}, outs[kLayers] = {width, width, width, n_out};
    int64_t off = 0;
    for (int l = 0; l < kLayers; ++l) {
        m->in_[l] = ins[l];
        m->out_[l] = outs[l];
        m->offW[l] = off;
        off += (int64_t)ins[l] * outs[l];
        m->offb[l] = off;
        off += outs[l];
    }
    m->np = off;
    std::vector<float> p(off, 0.f);
    uint64_t s = seed;
    for (int l = 0; l < kLayers; ++l) {
        const double a = std::sqrt(6.0 / (double)(ins[l] + outs[l]));
        for (int64_t i = 0; i < (int64_t)ins[l] * outs[l]; ++i) p[m->offW[l] + i] = (float)((2 * uniform01(s) - 1) * a);
    }
    bool ok = dalloc(m->P, off) && dalloc(m->G, off) && dalloc(m->Mm, off) && dalloc(m->Vv, off) &&
              dalloc(m->Ph, off) && dalloc(m->loss, 1);
    if (!ok) {
        gsis_mlp_destroy(m);
        return GSIS_E_OOM;
    }
    // set-up of the allocation-free entry point on this device (a failed lookup is reported by that call)
    m->scratch = scratch_address(device);
    *out = m;
    return gsis_mlp_set_params(m, p.data());
}

void gsis_mlp_destroy(gsis_mlp_t *m)
{
    if (!m) return;
    (void)hipSetDevice(m->device);
    if (m->st) (void)hipStreamSynchronize(m->st);
    else (void)hipDeviceSynchronize();
    free_batch(m);
    dfree(m->P);
    dfree(m->G);
    dfree(m->Mm);
    dfree(m->Vv);
    dfree(m->Ph);
    dfree(m->loss);
    delete m;
}

const char *gsis_mlp_last_error(gsis_mlp_t *m) { return m ? m->err.c_str() : "null handle"; }

int32_t gsis_mlp_set_stream(gsis_mlp_t *m, void *hip_stream)
{
    if (!m) return GSIS_E_ARG;
    m->st = (hipStream_t)hip_stream;
    return GSIS_OK;
}

int64_t gsis_mlp_num_params(gsis_mlp_t *m) { return m ? m->np : (int64_t)GSIS_E_ARG; }

int32_t gsis_mlp_get_params(gsis_mlp_t *m, float *params)
{
    if (!m || !params) return GSIS_E_ARG;
    (void)hipSetDevice(m->device);
    MCHECK(m, hipStreamSynchronize(m->st));
    MCHECK(m, hipMemcpy(params, m->P, m->np * sizeof(float), hipMemcpyDeviceToHost));
    return GSIS_OK;
}

int32_t gsis_mlp_set_params(gsis_mlp_t *m, const float *params)
{
    if (!m || !params) return GSIS_E_ARG;
    (void)hipSetDevice(m->device);
    MCHECK(m, hipStreamSynchronize(m->st));
    MCHECK(m, hipMemcpy(m->P, params, m->np * sizeof(float), hipMemcpyHostToDevice));
    MCHECK(m, hipMemset(m->Mm, 0, m->np * sizeof(float)));
    MCHECK(m, hipMemset(m->Vv, 0, m->np * sizeof(float)));
    hipLaunchKernelGGL(k_to_bf16, dim3((m->np + 255) / 256), dim3(256), 0, m->st, m->np, m->P, m->Ph);
    MCHECK(m, hipStreamSynchronize(m->st));
    m->adam_t = 0;
    return GSIS_OK;
}

int32_t gsis_mlp_forward(gsis_mlp_t *m, int64_t n, const float *x, float *y)
{
    if (!m || !y) return GSIS_E_ARG;
    int32_t rc = check_rows(m, n, x);
    if (rc != GSIS_OK) return rc;
    (void)hipSetDevice(m->device);
    if ((rc = upload_rows(m, n, x, nullptr)) != GSIS_OK) return rc;
    forward(m, (int)n);
    MCHECK(m, hipMemcpyAsync(y, m->Y, n * m->n_out * sizeof(float), hipMemcpyDeviceToHost, m->st));
    MCHECK(m, hipStreamSynchronize(m->st));
    return GSIS_OK;
}

int32_t gsis_mlp_forward_noalloc(gsis_mlp_t *m, int64_t n, const float *x, float *y)
{
    if (!m) return GSIS_E_ARG;
    if (n < 0 || n > INT_MAX) return fail(m, GSIS_E_ARG, "gsis_mlp_forward_noalloc: row count out of range");
    if (n > 0 && (!x || !y)) return fail(m, GSIS_E_ARG, "gsis_mlp_forward_noalloc: null input or output");
    if (!m->scratch)
        return fail(m, GSIS_E_DEVICE, "gsis_mlp_forward_noalloc: the scratch array has no address on this device");
    // two hidden buffers of `rows` rows each; larger batches go through in consecutive chunks of rows (rows are
    // independent, so the result does not depend on the chunking)
    const int64_t per_row = 2 * (int64_t)m->width;
    if (per_row > kScratchFloats)
        return fail(m, GSIS_E_ARG, "gsis_mlp_forward_noalloc: width " + std::to_string(m->width) +
                                       " needs more than the " + std::to_string(kScratchFloats * 4) +
                                       "-byte scratch array for one row");
    const int64_t rows = kScratchFloats / per_row;
    MCHECK(m, hipSetDevice(m->device));
    float *H0 = m->scratch, *H1 = m->scratch + rows * m->width;
    for (int64_t r0 = 0; r0 < n; r0 += rows) {
        const int nr = (int)std::min<int64_t>(rows, n - r0);
        forward_rows(m, nr, x + r0 * m->n_in, H0, H1, H0, y + r0 * m->n_out);
    }
    MCHECK(m, hipGetLastError());
    return GSIS_OK;
}

int32_t gsis_mlp_loss_grad(gsis_mlp_t *m, int64_t n, const float *x, const float *t, double *loss, float *grad)
{
    if (!m || !t) return GSIS_E_ARG;
    int32_t rc = check_rows(m, n, x);
    if (rc != GSIS_OK) return rc;
    (void)hipSetDevice(m->device);
    if ((rc = upload_rows(m, n, x, t)) != GSIS_OK) return rc;
    forward(m, (int)n);
    backward(m, (int)n);
    if (loss) MCHECK(m, hipMemcpyAsync(loss, m->loss, sizeof(double), hipMemcpyDeviceToHost, m->st));
    if (grad) MCHECK(m, hipMemcpyAsync(grad, m->G, m->np * sizeof(float), hipMemcpyDeviceToHost, m->st));
    MCHECK(m, hipStreamSynchronize(m->st));
    return GSIS_OK;
}

int32_t gsis_mlp_adam_step(gsis_mlp_t *m, const gsis_mlp_train_opts *o, int64_t n, const float *x, const float *t,
                           double *loss)
{
    if (!m || !o || !t) return GSIS_E_ARG;
    int32_t rc = check_rows(m, n, x);
    if (rc != GSIS_OK) return rc;
    (void)hipSetDevice(m->device);
    if ((rc = upload_rows(m, n, x, t)) != GSIS_OK) return rc;
    forward(m, (int)n);
    backward(m, (int)n);
    adam(m, o);
    if (loss) MCHECK(m, hipMemcpyAsync(loss, m->loss, sizeof(double), hipMemcpyDeviceToHost, m->st));
    MCHECK(m, hipStreamSynchronize(m->st));
    return GSIS_OK;
}

int32_t gsis_mlp_train(gsis_mlp_t *m, int64_t n, const float *x, const float *t, const gsis_mlp_train_opts *o,
                       double *final_loss)
{
    if (!m || !o || !t) return GSIS_E_ARG;
    int32_t rc = check_rows(m, n, x);
    if (rc != GSIS_OK) return rc;
    if (o->epochs < 0 || o->batch < 1 || !(o->lr > 0)) return fail(m, GSIS_E_ARG, "gsis_mlp_train: invalid options");
    (void)hipSetDevice(m->device);
    float *Xall = nullptr, *Tall = nullptr;
    struct Guard {
        float *&a, *&b;
        ~Guard()
        {
            dfree(a);
            dfree(b);
        }
    } guard{Xall, Tall};
    if (!(dalloc(Xall, n * m->n_in) && dalloc(Tall, n * m->n_out)))
        return fail(m, GSIS_E_OOM, "gsis_mlp_train: device allocation failed");
    MCHECK(m, hipMemcpyAsync(Xall, x, n * m->n_in * sizeof(float), hipMemcpyHostToDevice, m->st));
    MCHECK(m, hipMemcpyAsync(Tall, t, n * m->n_out * sizeof(float), hipMemcpyHostToDevice, m->st));
    return train_device(m, n, Xall, Tall, o, final_loss);
}

int32_t gsis_ws_fit_norm(int64_t n, int32_t n_in, const double *x, int32_t n_out, const double *t,
                         gsis_ws_norm *norm)
{
    if (n <= 0 || !x || !t || !norm || n_in < 1 || n_in > 64 || n_out < 1 || n_out > 64) return GSIS_E_ARG;
    std::memset(norm, 0, sizeof(*norm));
    norm->n_in = n_in;
    norm->n_out = n_out;
    auto stats = [&](const double *a, int k, double *mean, double *scale) {
        for (int j = 0; j < k; ++j) {
            double s1 = 0;
            for (int64_t i = 0; i < n; ++i) s1 += a[i * k + j];
            const double mu = s1 / (double)n;
            double s2 = 0;
            for (int64_t i = 0; i < n; ++i) s2 += (a[i * k + j] - mu) * (a[i * k + j] - mu);
            mean[j] = mu;
            scale[j] = std::sqrt(s2 / (double)n) + 1e-12;
        }
    };
    stats(x, n_in, norm->x_mean, norm->x_scale);
    stats(t, n_out, norm->y_mean, norm->y_scale);
    return GSIS_OK;
}

int32_t gsis_ws_train(gsis_mlp_t *m, const gsis_ws_norm *norm, int64_t n, const double *x, const double *t,
                      const gsis_mlp_train_opts *o, double *final_loss)
{
    if (!m || !o || !t) return GSIS_E_ARG;
    int32_t rc = check_rows(m, n, x);
    if (rc != GSIS_OK) return rc;
    if (o->epochs < 0 || o->batch < 1 || !(o->lr > 0)) return fail(m, GSIS_E_ARG, "gsis_ws_train: invalid options");
    (void)hipSetDevice(m->device);
    double *dn = nullptr, *raw = nullptr;
    float *Xall = nullptr, *Tall = nullptr;
    struct Guard {
        double *&a, *&b;
        float *&c, *&d;
        ~Guard()
        {
            dfree(a);
            dfree(b);
            dfree(c);
            dfree(d);
        }
    } guard{dn, raw, Xall, Tall};
    if ((rc = upload_norm(m, norm, dn)) != GSIS_OK) return rc;
    const int64_t k = std::max(m->n_in, m->n_out);
    if (!(dalloc(raw, n * k) && dalloc(Xall, n * m->n_in) && dalloc(Tall, n * m->n_out)))
        return fail(m, GSIS_E_OOM, "gsis_ws_train: device allocation failed");
    MCHECK(m, hipMemcpyAsync(raw, x, n * m->n_in * sizeof(double), hipMemcpyHostToDevice, m->st));
    gsis::launch_standardize(raw, dn, dn + 64, Xall, n, m->n_in, m->st);
    MCHECK(m, hipStreamSynchronize(m->st));
    MCHECK(m, hipMemcpyAsync(raw, t, n * m->n_out * sizeof(double), hipMemcpyHostToDevice, m->st));
    gsis::launch_standardize(raw, dn + 128, dn + 192, Tall, n, m->n_out, m->st);
    MCHECK(m, hipStreamSynchronize(m->st));
    return train_device(m, n, Xall, Tall, o, final_loss);
}

int32_t gsis_ws_predict(gsis_mlp_t *m, const gsis_ws_norm *norm, int64_t n, const double *x, double *y)
{
    if (!m || !y) return GSIS_E_ARG;
    int32_t rc = check_rows(m, n, x);
    if (rc != GSIS_OK) return rc;
    (void)hipSetDevice(m->device);
    double *dn = nullptr, *raw = nullptr;
    struct Guard {
        double *&a, *&b;
        ~Guard()
        {
            dfree(a);
            dfree(b);
        }
    } guard{dn, raw};
    if ((rc = upload_norm(m, norm, dn)) != GSIS_OK) return rc;
    if (!ensure_batch(m, n) || !dalloc(raw, n * std::max(m->n_in, m->n_out)))
        return fail(m, GSIS_E_OOM, "gsis_ws_predict: device allocation failed");
    MCHECK(m, hipMemcpyAsync(raw, x, n * m->n_in * sizeof(double), hipMemcpyHostToDevice, m->st));
    gsis::launch_standardize(raw, dn, dn + 64, m->X, n, m->n_in, m->st);
    forward(m, (int)n);
    hipLaunchKernelGGL(k_destandardize, dim3((unsigned)((n * m->n_out + 255) / 256)), dim3(256), 0, m->st, m->Y,
                       dn + 128, dn + 192, raw, n, m->n_out);
    MCHECK(m, hipMemcpyAsync(y, raw, n * m->n_out * sizeof(double), hipMemcpyDeviceToHost, m->st));
    MCHECK(m, hipStreamSynchronize(m->st));
    return GSIS_OK;
}

// file: 8-byte tag "GSISMLP1", int32 n_in, width, n_out, bf16, int64 parameter count, FP32 parameters, norm
int32_t gsis_ws_save(gsis_mlp_t *m, const gsis_ws_norm *norm, const char *path)
{
    if (!m || !norm || !path) return GSIS_E_ARG;
    if (norm->n_in != m->n_in || norm->n_out != m->n_out) return fail(m, GSIS_E_ARG, "gsis_ws_save: norm dimensions");
    std::vector<float> P(m->np);
    int32_t rc = gsis_mlp_get_params(m, P.data());
    if (rc != GSIS_OK) return rc;
    FILE *fp = fopen(path, "wb");
    if (!fp) return fail(m, GSIS_E_ARG, std::string("gsis_ws_save: cannot open ") + path);
    const int32_t dims[4] = {m->n_in, m->width, m->n_out, m->bf16 ? 1 : 0};
    const int64_t np = m->np;
    bool ok = fwrite("GSISMLP1", 1, 8, fp) == 8 && fwrite(dims, sizeof(dims), 1, fp) == 1 &&
              fwrite(&np, sizeof(np), 1, fp) == 1 && fwrite(P.data(), sizeof(float), np, fp) == (size_t)np &&
              fwrite(norm, sizeof(*norm), 1, fp) == 1;
    ok = (fclose(fp) == 0) && ok;
    return ok ? GSIS_OK : fail(m, GSIS_E_ARG, "gsis_ws_save: write failed");
}

int32_t gsis_ws_load(gsis_mlp_t *m, gsis_ws_norm *norm, const char *path)
{
    if (!m || !norm || !path) return GSIS_E_ARG;
    FILE *fp = fopen(path, "rb");
    if (!fp) return fail(m, GSIS_E_ARG, std::string("gsis_ws_load: cannot open ") + path);
    char tag[8];
    int32_t dims[4];
    int64_t np = 0;
    bool ok = fread(tag, 1, 8, fp) == 8 && memcmp(tag, "GSISMLP1", 8) == 0 && fread(dims, sizeof(dims), 1, fp) == 1 &&
              fread(&np, sizeof(np), 1, fp) == 1;
    ok = ok && dims[0] == m->n_in && dims[1] == m->width && dims[2] == m->n_out && np == m->np;
    std::vector<float> P(ok ? np : 0);
    gsis_ws_norm nm;
    ok = ok && fread(P.data(), sizeof(float), np, fp) == (size_t)np && fread(&nm, sizeof(nm), 1, fp) == 1;
    fclose(fp);
    if (!ok) return fail(m, GSIS_E_ARG, "gsis_ws_load: not a network file of this handle's dimensions");
    int32_t rc = gsis_mlp_set_params(m, P.data());
    if (rc != GSIS_OK) return rc;
    *norm = nm;
    return GSIS_OK;
}

}  // extern "C"
