// mlp.hip -- learned refinement flags: per-block features, a 512-128-128-1 MLP
// on bf16 MFMA (fp32 accumulate), its backward pass and Adam.
//
// The network predicts, from a block's primitive variables, whether the plain
// refinement criterion (Loehner density/velocity estimator with div V < 0 in
// the Earth/CME windows, paper Sect. 3.2) will ask for refinement of that
// block; the plain criterion stays the judge and the fallback.
//
// Rounding points (the CPU reference follows the same ones): inputs X, the
// weights W1, W2, w3 and the hidden activations H1 = relu(Z1), H2 = relu(Z2)
// are bf16 (round to nearest even from fp32); products accumulate in fp32; in
// the backward pass dZ2 and dZ1 enter the GEMMs as bf16 while the bias
// gradients sum the fp32 values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "devmem.h"
#include "kernels.h"
#include "mlp.h"

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
#define DEV_EPI __device__ __forceinline__

// ---------------------------------------------------------------------------
// features: 8 primitives x 4^3 patch means, [prim][k][j][i]
// ---------------------------------------------------------------------------
template <int BI, int BJ, int BK>
__global__ void __launch_bounds__(256) k_features(KArgs a, const int *items, const int *nitems_ptr, float *raw,
                                                  const float *mean, const float *istd, uint16_t *xb)
{
    using S = Shape<BI, BJ, BK>;
    constexpr int PI = BI / 4, PJ = BJ / 4, PK = BK / 4;
    const int n = *nitems_ptr;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int slot = items[it];
        const int t = threadIdx.x;
        if (t < 64) {
            const int pi = t & 3, pj = (t >> 2) & 3, pk = t >> 4;
            double sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int k = pk * PK; k < (pk + 1) * PK; ++k)
                for (int j = pj * PJ; j < (pj + 1) * PJ; ++j)
                    for (int i = pi * PI; i < (pi + 1) * PI; ++i) {
                        double u[8], w[8];
                        for (int v = 0; v < 8; ++v)
                            u[v] = a.U[((size_t)slot * a.nv + v) * S::NC + i + BI * (j + BJ * k)];
                        cons_to_prim<true>(u, w, a.gas);
                        for (int v = 0; v < 8; ++v) sum[v] += w[v];
                    }
            const double inv = 1.0 / (PI * PJ * PK);
            for (int v = 0; v < 8; ++v) {
                double m = sum[v] * inv;
                if (v == 0 || v == 4) m = log10(m);
                const float f = (float)m;
                const int idx = v * 64 + t;
                if (raw) raw[(size_t)it * IC_MLP_IN + idx] = f;
                if (xb) xb[(size_t)it * IC_MLP_IN + idx] = f2bf((f - mean[idx]) * istd[idx]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// GEMM: C = A B (+ bias, relu), bf16 operands, fp32 accumulate on gfx950's
// v_mfma_f32_16x16x32_bf16.  A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn].
// A work-group of 4 waves computes a 64x64 tile of C, each wave a 32x32
// quarter as 2x2 MFMA blocks of 16x16.  K advances in MFMA steps of 32 (the
// order in which they accumulate), staged through LDS four steps (128 k) at
// a time: As[m][k] and Bt[n][k] with k contiguous, so that a lane's MFMA
// operand -- row (A) or column (B) l % 16 and eight consecutive k,
// 8 (l / 16) + 0..7 -- is one 16-byte LDS read (rows padded by 8 bf16 to
// spread them over the banks).  Each thread moves 16-byte pieces (eight
// elements along whichever index is contiguous in memory) with one global
// load each; the next stage's loads are in flight while the MFMAs of the
// current one run, from the other of two LDS buffers.  The accumulator holds
// column l % 16 and rows 4 (l / 16) + 0..3 of a block.
// Split K (gridDim.z > 1, weight gradients with K = the batch rows): each
// z-slice accumulates its share of the k-steps and writes fp32 partials
// P[z][m][n]; k_gemm_reduce sums them in slice order (deterministic) and
// applies the epilogue.
// ---------------------------------------------------------------------------
struct GemmArgs {
    const uint16_t *A;
    long sam, sak;
    const uint16_t *B;
    long sbk, sbn;
    int M, N, K;
    const float *bias;
    int relu;
    float *Cf;
    uint16_t *Cb;
    long ldc;
    float *P;                 // split-K partials [gridDim.z][M][N] (gridDim.z > 1)
};

DEV_EPI void gemm_store(const GemmArgs &g, int m, int n, float v)
{
    if (g.bias) v += g.bias[n];
    if (g.relu) v = v > 0.f ? v : 0.f;
    if (g.Cf) g.Cf[(long)m * g.ldc + n] = v;
    if (g.Cb) g.Cb[(long)m * g.ldc + n] = f2bf(v);
}

constexpr int GEMM_KS = 128;               // k per LDS stage (four MFMA steps)
constexpr int GEMM_KP = GEMM_KS + 8;       // padded LDS row, bf16

// The 16-byte pieces of one stage of a 64-row operand tile X(r, k) (r = m of
// A or n of B): piece e of thread tid.  kc: X is contiguous along k (pieces
// run along k, 16 per row of the stage); else along r (8 per k-row).
// Pieces outside 0 <= r < R or k < K are zero.
DEV_EPI void tile_load(const uint16_t *X, long sr, long sk, bool kc, int r0, int R, int kb, int K, int tid,
                       uint4 *out)
{
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int c = e * 256 + tid;
        const int r = kc ? c >> 4 : (c & 7) * 8, k = kc ? (c & 15) * 8 : c >> 3;
        const int gr = r0 + r, gk = kb + k;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (gr < R && gk < K) v = *(const uint4 *)(X + (long)gr * sr + (long)gk * sk);
        out[e] = v;
    }
}

DEV_EPI void tile_store(uint16_t *L, bool kc, int tid, const uint4 *in)
{
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int c = e * 256 + tid;
        if (kc) {
            *(uint4 *)&L[(c >> 4) * GEMM_KP + (c & 15) * 8] = in[e];
        } else {                                  // eight rows, one k: transposed into LDS
            const int r = (c & 7) * 8, k = c >> 3;
            const uint32_t w[4] = {in[e].x, in[e].y, in[e].z, in[e].w};
#pragma unroll
            for (int i = 0; i < 8; ++i) L[(r + i) * GEMM_KP + k] = (uint16_t)(w[i >> 1] >> (16 * (i & 1)));
        }
    }
}

__global__ void __launch_bounds__(256) k_gemm(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[2][64 * GEMM_KP];
    __shared__ __attribute__((aligned(16))) uint16_t Bt[2][64 * GEMM_KP];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const int nstep = (g.K + 31) / 32;
    const int s0 = (int)((long)nstep * blockIdx.z / gridDim.z), s1 = (int)((long)nstep * (blockIdx.z + 1) / gridDim.z);
    // A as X(m, k): contiguous along k when sak == 1; B as X(n, k): along k when sbk == 1
    const bool a_k = g.sak == 1, b_k = g.sbk == 1;
    const long ar = g.sam, ak = g.sak, br = g.sbn, bk = g.sbk;
    float4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
    const int kend = s1 * 32;
    uint4 ra[4], rb[4];
    int kb = s0 * 32;
    if (kb < kend) {
        tile_load(g.A, ar, ak, a_k, m0, g.M, kb, g.K, tid, ra);
        tile_load(g.B, br, bk, b_k, n0, g.N, kb, g.K, tid, rb);
    }
    for (int buf = 0; kb < kend; kb += GEMM_KS, buf ^= 1) {
        // the buffer written here was last read two stages ago, before the
        // barrier of the previous stage
        tile_store(As[buf], a_k, tid, ra);
        tile_store(Bt[buf], b_k, tid, rb);
        __syncthreads();
        if (kb + GEMM_KS < kend) {
            tile_load(g.A, ar, ak, a_k, m0, g.M, kb + GEMM_KS, g.K, tid, ra);
            tile_load(g.B, br, bk, b_k, n0, g.N, kb + GEMM_KS, g.K, tid, rb);
        }
        const int nk = (kend - kb < GEMM_KS ? kend - kb : GEMM_KS) / 32;
        for (int kk = 0; kk < nk; ++kk) {
            bf16x8_t a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8_t *)&As[buf][(wm + 16 * i + r) * GEMM_KP + kk * 32 + kq];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = *(const bf16x8_t *)&Bt[buf][(wn + 16 * j + r) * GEMM_KP + kk * 32 + kq];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int m = m0 + wm + 16 * i + (lane >> 4) * 4 + t, n = n0 + wn + 16 * j + r;
                if (m < g.M && n < g.N) {
                    if (gridDim.z > 1) g.P[((long)blockIdx.z * g.M + m) * g.N + n] = acc[i][j][t];
                    else gemm_store(g, m, n, acc[i][j][t]);
                }
            }
}

// C = the sum of the split-K partials in slice order, then bias / relu / stores
__global__ void k_gemm_reduce(GemmArgs g, int nz)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)g.M * g.N) return;
    float v = 0.f;
    for (int z = 0; z < nz; ++z) v += g.P[(long)z * g.M * g.N + q];
    gemm_store(g, (int)(q / g.N), (int)(q % g.N), v);
}

// logit, probability and (training) the weighted-BCE gradient per row:
// z = sum_j H2[j] w3[j] + b3 (fp32, j ascending); dl/dz = (s (pw y + 1 - y) - pw y) / n
__global__ void k_head(const uint16_t *H2, const uint16_t *w3, const float *b3, int n, const uint8_t *y,
                       float pw, float *z, float *prob, float *dz, float *loss)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    float s = 0.f;
    for (int j = 0; j < IC_MLP_HID; ++j) s += bf2f(H2[(long)b * IC_MLP_HID + j]) * bf2f(w3[j]);
    s += b3[0];
    const float p = 1.f / (1.f + expf(-s));
    if (z) z[b] = s;
    if (prob) prob[b] = p;
    if (y) {
        const float yy = (float)y[b];
        dz[b] = (p * (pw * yy + 1.f - yy) - pw * yy) / (float)n;
        // stable log-sigmoid terms
        const float lsp = s >= 0.f ? -log1pf(expf(-s)) : s - log1pf(expf(s));     // log p
        const float lsn = s >= 0.f ? -s - log1pf(expf(-s)) : -log1pf(expf(s));   // log (1 - p)
        loss[b] = -(pw * yy * lsp + (1.f - yy) * lsn);
    }
}

// dZ2 = dz w3 [H2 > 0] (fp32 and bf16 copies)
__global__ void k_back2(const float *dz, const uint16_t *w3, const uint16_t *H2, int n, float *dZ2, uint16_t *dZ2b)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)n * IC_MLP_HID) return;
    const int b = (int)(q / IC_MLP_HID), j = (int)(q % IC_MLP_HID);
    const float v = bf2f(H2[q]) > 0.f ? dz[b] * bf2f(w3[j]) : 0.f;
    dZ2[q] = v;
    dZ2b[q] = f2bf(v);
}

// dZ1 = dH1 [H1 > 0]
__global__ void k_mask(const float *dH, const uint16_t *H, long count, float *dZ, uint16_t *dZb)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const float v = bf2f(H[q]) > 0.f ? dH[q] : 0.f;
    dZ[q] = v;
    dZb[q] = f2bf(v);
}

// column sums out[j] = sum_b w[b] * M[b][j] (w = NULL: plain sums), fp32, in
// two levels: chunk c of the rows (gridDim.y chunks, rows ascending within a
// chunk) into P[c][j], then the chunks in order (k_colsum_reduce)
__global__ void k_colsum(const float *Mf, const uint16_t *Mb, const float *w, int n, int ncol, float *P)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ncol) return;
    const int c = blockIdx.y, nc = gridDim.y;
    const int b0 = (int)((long)n * c / nc), b1 = (int)((long)n * (c + 1) / nc);
    float s = 0.f;
    for (int b = b0; b < b1; ++b) {
        const float m = Mf ? Mf[(long)b * ncol + j] : bf2f(Mb[(long)b * ncol + j]);
        s += w ? w[b] * m : m;
    }
    P[(long)c * ncol + j] = s;
}

__global__ void k_colsum_reduce(const float *P, int nc, int ncol, float *out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ncol) return;
    float s = 0.f;
    for (int c = 0; c < nc; ++c) s += P[(long)c * ncol + j];
    out[j] = s;
}

// sum of the n per-row losses in fp64 (fixed order: thread-strided, then a
// pairwise tree) into out[slot]
__global__ void __launch_bounds__(256) k_loss_sum(const float *loss, int n, double *out, long slot)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < n; b += 256) s += (double)loss[b];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[slot] = sh[0];
}

__global__ void k_adam(float *w, uint16_t *wb, const float *g, float *m1, float *m2, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float gg = g[q];
    m1[q] = b1 * m1[q] + (1.f - b1) * gg;
    m2[q] = b2 * m2[q] + (1.f - b2) * gg * gg;
    const float mh = m1[q] / c1, vh = m2[q] / c2;
    w[q] -= lr * mh / (sqrtf(vh) + eps);
    if (wb) wb[q] = f2bf(w[q]);
}

__global__ void k_to_bf16(const float *x, uint16_t *y, long n)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) y[q] = f2bf(x[q]);
}

// normalised bf16 inputs from raw fp32 features
__global__ void k_normalise(const float *raw, const float *mean, const float *istd, long n, uint16_t *xb)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n * IC_MLP_IN) return;
    const int f = (int)(q % IC_MLP_IN);
    xb[q] = f2bf((raw[q] - mean[f]) * istd[f]);
}

// 1 / std per input (fp32 division, correctly rounded as on the host)
__global__ void k_istd(const float *std, float *istd)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < IC_MLP_IN) istd[f] = 1.0f / std[f];
}

// minibatch gather: rows order[b0 + q] of the normalised inputs and labels
__global__ void k_gather(const uint16_t *xall, const uint8_t *yall, const long *order, long b0, int B, uint16_t *xb,
                         uint8_t *yb)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)B * IC_MLP_IN) return;
    const int r = (int)(q / IC_MLP_IN), f = (int)(q % IC_MLP_IN);
    const long row = order[b0 + r];
    xb[q] = xall[row * IC_MLP_IN + f];
    if (f == 0) yb[r] = yall[row];
}

// learned flags: p >= threshold -> refine, else coarsen-eligible
__global__ void k_prob_flags(const float *prob, const int *items, int n, float threshold, int8_t *flags)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) flags[items[q]] = prob[q] >= threshold ? 1 : -1;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

// Split K only when a workspace is given (the weight gradients): enough
// slices for ~256 work-groups, each at least 4 k-steps; the workspace holds
// GEMM_SPLIT_MAX x M x N floats.
constexpr int GEMM_SPLIT_MAX = 32;

void gemm(hipStream_t s, const uint16_t *A, long sam, long sak, const uint16_t *B, long sbk, long sbn, int M, int N,
          int K, const float *bias, int relu, float *Cf, uint16_t *Cb, long ldc, float *work = nullptr)
{
    // the stage loads move 16-byte pieces along the contiguous index of each
    // operand: a unit stride, the other stride and that index's extent
    // multiples of 8, 16-byte aligned bases (every call of this file)
    const bool a_ok = (sak == 1 && sam % 8 == 0 && K % 8 == 0) || (sam == 1 && sak % 8 == 0 && M % 8 == 0);
    const bool b_ok = (sbk == 1 && sbn % 8 == 0 && K % 8 == 0) || (sbn == 1 && sbk % 8 == 0 && N % 8 == 0);
    if (!a_ok || !b_ok || ((uintptr_t)A & 15) || ((uintptr_t)B & 15))
        throw std::runtime_error("gemm: operand layout not supported by the staged loads");
    GemmArgs g{A, sam, sak, B, sbk, sbn, M, N, K, bias, relu, Cf, Cb, ldc, work};
    const int tiles = ((N + 63) / 64) * ((M + 63) / 64), nstep = (K + 31) / 32;
    int nz = 1;
    if (work && tiles < 256) nz = std::max(1, std::min({GEMM_SPLIT_MAX, nstep / 4, (256 + tiles - 1) / tiles}));
    dim3 grid((N + 63) / 64, (M + 63) / 64, nz);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g);
    if (nz > 1)
        hipLaunchKernelGGL(k_gemm_reduce, dim3(((long)M * N + 255) / 256), dim3(256), 0, s, g, nz);
}

// column sums through the workspace (COLSUM_CHUNKS x ncol floats)
constexpr int COLSUM_CHUNKS = 64;

void colsum(hipStream_t s, const float *Mf, const uint16_t *Mb, const float *w, int n, int ncol, float *out,
            float *work)
{
    const int nc = std::max(1, std::min(COLSUM_CHUNKS, n / 32));
    hipLaunchKernelGGL(k_colsum, dim3((ncol + 127) / 128, nc), dim3(128), 0, s, Mf, Mb, w, n, ncol, work);
    hipLaunchKernelGGL(k_colsum_reduce, dim3((ncol + 127) / 128), dim3(128), 0, s, (const float *)work, nc, ncol, out);
}

template <class T>
struct Buf {
    T *p = nullptr;
    size_t n = 0;
    explicit Buf(size_t count = 0) { alloc(count); }
    void alloc(size_t count)
    {
        dev_free(p);
        p = nullptr;
        n = count;
        if (count && !(p = (T *)dev_malloc(count * sizeof(T)))) throw std::runtime_error("device allocation failed");
    }
    ~Buf() { dev_free(p); }
    Buf(const Buf &) = delete;
    Buf &operator=(const Buf &) = delete;
};

}  // namespace

MlpDevice::MlpDevice() = default;

MlpDevice::~MlpDevice()
{
    for (void *q : {(void *)w, (void *)wb, (void *)mean, (void *)istd, (void *)xb, (void *)h1, (void *)h2,
                    (void *)prob, (void *)flags_tmp})
        dev_free(q);
}

void MlpDevice::set(const float *params, const float *mean_h, const float *std_h)
{
    if (!w) {
        w = (float *)dev_malloc(IC_MLP_NPARAM * sizeof(float));
        wb = (uint16_t *)dev_malloc(IC_MLP_NPARAM * sizeof(uint16_t));
        mean = (float *)dev_malloc(IC_MLP_IN * sizeof(float));
        istd = (float *)dev_malloc(IC_MLP_IN * sizeof(float));
        if (!w || !wb || !mean || !istd) throw std::runtime_error("device allocation failed");
    }
    std::vector<float> is(IC_MLP_IN);
    for (int f = 0; f < IC_MLP_IN; ++f) is[f] = 1.0f / std_h[f];
    if (hipMemcpy(w, params, IC_MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mean, mean_h, IC_MLP_IN * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(istd, is.data(), IC_MLP_IN * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        throw std::runtime_error("hipMemcpy failed");
    hipLaunchKernelGGL(k_to_bf16, dim3((IC_MLP_NPARAM + 255) / 256), dim3(256), 0, 0, w, wb, (long)IC_MLP_NPARAM);
    if (hipDeviceSynchronize() != hipSuccess) throw std::runtime_error("device error");
    ready = true;
}

void MlpDevice::reserve(int n)
{
    if (n <= cap) return;
    for (void *q : {(void *)xb, (void *)h1, (void *)h2, (void *)prob}) dev_free(q);
    xb = h1 = h2 = nullptr;
    prob = nullptr;
    cap = n + n / 2 + 64;
    xb = (uint16_t *)dev_malloc((size_t)cap * IC_MLP_IN * sizeof(uint16_t));
    h1 = (uint16_t *)dev_malloc((size_t)cap * IC_MLP_HID * sizeof(uint16_t));
    h2 = (uint16_t *)dev_malloc((size_t)cap * IC_MLP_HID * sizeof(uint16_t));
    prob = (float *)dev_malloc((size_t)cap * sizeof(float));
    if (!xb || !h1 || !h2 || !prob) throw std::runtime_error("device allocation failed");
}

// forward pass over n rows of xb (already filled) -> prob
void MlpDevice::forward(hipStream_t s, int n)
{
    const uint16_t *W1 = wb + IC_MLP_OFF_W1, *W2 = wb + IC_MLP_OFF_W2, *w3 = wb + IC_MLP_OFF_W3;
    gemm(s, xb, IC_MLP_IN, 1, W1, IC_MLP_HID, 1, n, IC_MLP_HID, IC_MLP_IN, w + IC_MLP_OFF_B1, 1, nullptr, h1,
         IC_MLP_HID);
    gemm(s, h1, IC_MLP_HID, 1, W2, IC_MLP_HID, 1, n, IC_MLP_HID, IC_MLP_HID, w + IC_MLP_OFF_B2, 1, nullptr, h2,
         IC_MLP_HID);
    hipLaunchKernelGGL(k_head, dim3((n + 255) / 256), dim3(256), 0, s, h2, w3, w + IC_MLP_OFF_B3, n,
                       (const uint8_t *)nullptr, 0.f, (float *)nullptr, prob, (float *)nullptr, (float *)nullptr);
}

void mlp_features(hipStream_t s, const KArgs &a, int bi, int bj, int bk, const int *items,
                  const int *nitems, int n, float *raw, const float *mean, const float *istd, uint16_t *xb)
{
    const dim3 g(std::max(1, std::min(n, 16384)));
#define IC_INSTANTIATE(BI, BJ, BK)                                                                      \
    if (bi == BI && bj == BJ && bk == BK) {                                                            \
        hipLaunchKernelGGL((k_features<BI, BJ, BK>), g, dim3(256), 0, s, a, items, nitems, raw, mean,   \
                           istd, xb);                                                                   \
        return;                                                                                        \
    }
#include "shapes.inc"
#undef IC_INSTANTIATE
}

void mlp_prob_flags(hipStream_t s, const float *prob, const int *items, int n, float threshold, int8_t *flags)
{
    hipLaunchKernelGGL(k_prob_flags, dim3((n + 255) / 256), dim3(256), 0, s, prob, items, n, threshold, flags);
}

// One forward + backward pass on n rows: gradients (fp32, params layout) and mean loss.
// X: normalised fp32 inputs (converted to bf16 here), params: fp32 master weights.
// Workspace of fwd_bwd: split-K partials of the largest weight gradient, or
// the chunked column sums
constexpr size_t FWD_BWD_WORK = (size_t)GEMM_SPLIT_MAX * IC_MLP_IN * IC_MLP_HID;

static void fwd_bwd(hipStream_t s, int n, const uint16_t *Xb, const uint8_t *y, float pw, const float *w,
                    const uint16_t *wb, float *grad, float *loss_rows, Buf<uint16_t> &H1, Buf<uint16_t> &H2,
                    Buf<float> &dz, Buf<float> &dZ2, Buf<uint16_t> &dZ2b, Buf<float> &dH1, Buf<float> &dZ1,
                    Buf<uint16_t> &dZ1b, float *work)
{
    const uint16_t *W1 = wb + IC_MLP_OFF_W1, *W2 = wb + IC_MLP_OFF_W2, *w3 = wb + IC_MLP_OFF_W3;
    gemm(s, Xb, IC_MLP_IN, 1, W1, IC_MLP_HID, 1, n, IC_MLP_HID, IC_MLP_IN, w + IC_MLP_OFF_B1, 1, nullptr, H1.p,
         IC_MLP_HID);
    gemm(s, H1.p, IC_MLP_HID, 1, W2, IC_MLP_HID, 1, n, IC_MLP_HID, IC_MLP_HID, w + IC_MLP_OFF_B2, 1, nullptr,
         H2.p, IC_MLP_HID);
    hipLaunchKernelGGL(k_head, dim3((n + 255) / 256), dim3(256), 0, s, H2.p, w3, w + IC_MLP_OFF_B3, n, y, pw,
                       (float *)nullptr, (float *)nullptr, dz.p, loss_rows);
    // layer 3: dw3 = H2^T dz, db3 = sum dz
    colsum(s, nullptr, H2.p, dz.p, n, IC_MLP_HID, grad + IC_MLP_OFF_W3, work);
    colsum(s, dz.p, nullptr, nullptr, n, 1, grad + IC_MLP_OFF_B3, work);
    const long nh = (long)n * IC_MLP_HID;
    hipLaunchKernelGGL(k_back2, dim3((nh + 255) / 256), dim3(256), 0, s, dz.p, w3, H2.p, n, dZ2.p, dZ2b.p);
    colsum(s, dZ2.p, nullptr, nullptr, n, IC_MLP_HID, grad + IC_MLP_OFF_B2, work);
    // dW2 = H1^T dZ2   (M = 128 (k of layer 2), N = 128, K = n)
    gemm(s, H1.p, 1, IC_MLP_HID, dZ2b.p, IC_MLP_HID, 1, IC_MLP_HID, IC_MLP_HID, n, nullptr, 0, grad + IC_MLP_OFF_W2,
         nullptr, IC_MLP_HID, work);
    // dH1 = dZ2 W2^T   (B(k, j) = W2[j][k])
    gemm(s, dZ2b.p, IC_MLP_HID, 1, W2, 1, IC_MLP_HID, n, IC_MLP_HID, IC_MLP_HID, nullptr, 0, dH1.p, nullptr,
         IC_MLP_HID);
    hipLaunchKernelGGL(k_mask, dim3((nh + 255) / 256), dim3(256), 0, s, dH1.p, H1.p, nh, dZ1.p, dZ1b.p);
    colsum(s, dZ1.p, nullptr, nullptr, n, IC_MLP_HID, grad + IC_MLP_OFF_B1, work);
    // dW1 = X^T dZ1    (M = 512, N = 128, K = n)
    gemm(s, Xb, 1, IC_MLP_IN, dZ1b.p, IC_MLP_HID, 1, IC_MLP_IN, IC_MLP_HID, n, nullptr, 0, grad + IC_MLP_OFF_W1,
         nullptr, IC_MLP_HID, work);
}

void mlp_grad(const float *xnorm, const uint8_t *y, int n, float pw, const float *params, float *grad_out,
              float *loss_out)
{
    hipStream_t s = nullptr;
    Buf<float> x((size_t)n * IC_MLP_IN), w(IC_MLP_NPARAM), grad(IC_MLP_NPARAM), dz(n), loss(n), dZ2((size_t)n * IC_MLP_HID),
        dH1((size_t)n * IC_MLP_HID), dZ1((size_t)n * IC_MLP_HID);
    Buf<uint16_t> xb((size_t)n * IC_MLP_IN), wb(IC_MLP_NPARAM), H1((size_t)n * IC_MLP_HID), H2((size_t)n * IC_MLP_HID),
        dZ2b((size_t)n * IC_MLP_HID), dZ1b((size_t)n * IC_MLP_HID);
    Buf<uint8_t> yd(n);
    Buf<float> work(FWD_BWD_WORK);
    if (hipMemcpy(x.p, xnorm, (size_t)n * IC_MLP_IN * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(w.p, params, IC_MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(yd.p, y, n, hipMemcpyHostToDevice) != hipSuccess)
        throw std::runtime_error("hipMemcpy failed");
    hipLaunchKernelGGL(k_to_bf16, dim3(((long)n * IC_MLP_IN + 255) / 256), dim3(256), 0, s, x.p, xb.p,
                       (long)n * IC_MLP_IN);
    hipLaunchKernelGGL(k_to_bf16, dim3((IC_MLP_NPARAM + 255) / 256), dim3(256), 0, s, w.p, wb.p, (long)IC_MLP_NPARAM);
    fwd_bwd(s, n, xb.p, yd.p, pw, w.p, wb.p, grad.p, loss.p, H1, H2, dz, dZ2, dZ2b, dH1, dZ1, dZ1b, work.p);
    std::vector<float> lrow(n);
    if (hipMemcpy(grad_out, grad.p, IC_MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(lrow.data(), loss.p, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        throw std::runtime_error("hipMemcpy failed");
    double l = 0.0;
    for (int b = 0; b < n; ++b) l += lrow[b];
    *loss_out = (float)(l / n);
}

void mlp_train(const float *raw, const uint8_t *y, long n, const MlpHparams &hp, float *params, float *mean_out,
               float *std_out, float *loss_epochs)
{
    hipStream_t s = nullptr;
    // per-feature z-score statistics of the training set (fp64 on the host)
    std::vector<double> mu(IC_MLP_IN, 0.0), var(IC_MLP_IN, 0.0);
    for (long b = 0; b < n; ++b)
        for (int f = 0; f < IC_MLP_IN; ++f) mu[f] += raw[b * IC_MLP_IN + f];
    for (int f = 0; f < IC_MLP_IN; ++f) mu[f] /= (double)n;
    for (long b = 0; b < n; ++b)
        for (int f = 0; f < IC_MLP_IN; ++f) {
            const double d = raw[b * IC_MLP_IN + f] - mu[f];
            var[f] += d * d;
        }
    std::vector<float> mean_h(IC_MLP_IN), std_h(IC_MLP_IN), istd_h(IC_MLP_IN);
    for (int f = 0; f < IC_MLP_IN; ++f) {
        mean_h[f] = (float)mu[f];
        double sd = std::sqrt(var[f] / (double)n);
        if (!(sd > 1e-6)) sd = 1.0;
        std_h[f] = (float)sd;
        istd_h[f] = 1.0f / std_h[f];
    }
    long npos = 0;
    for (long b = 0; b < n; ++b) npos += y[b] ? 1 : 0;
    const float pw = hp.pos_weight > 0.f ? hp.pos_weight : (npos > 0 ? (float)(n - npos) / (float)npos : 1.f);
    const int B = hp.batch;
    Buf<float> rawd((size_t)n * IC_MLP_IN), mean(IC_MLP_IN), istd(IC_MLP_IN), w(IC_MLP_NPARAM), grad(IC_MLP_NPARAM),
        m1(IC_MLP_NPARAM), m2(IC_MLP_NPARAM), dz(B), loss(B), dZ2((size_t)B * IC_MLP_HID), dH1((size_t)B * IC_MLP_HID),
        dZ1((size_t)B * IC_MLP_HID);
    Buf<uint16_t> xall((size_t)n * IC_MLP_IN), xb((size_t)B * IC_MLP_IN), wb(IC_MLP_NPARAM), H1((size_t)B * IC_MLP_HID),
        H2((size_t)B * IC_MLP_HID), dZ2b((size_t)B * IC_MLP_HID), dZ1b((size_t)B * IC_MLP_HID);
    Buf<uint8_t> yall(n), yb(B);
    Buf<long> orderd(n);
    Buf<float> work(FWD_BWD_WORK);
    const long nbatch = n / B;
    Buf<double> lossacc(std::max(nbatch, 1L));           // per-minibatch loss sums, read once per epoch
    auto H2D = [](void *d, const void *h, size_t bytes) {
        if (hipMemcpy(d, h, bytes, hipMemcpyHostToDevice) != hipSuccess) throw std::runtime_error("hipMemcpy failed");
    };
    H2D(rawd.p, raw, (size_t)n * IC_MLP_IN * sizeof(float));
    H2D(mean.p, mean_h.data(), IC_MLP_IN * sizeof(float));
    H2D(istd.p, istd_h.data(), IC_MLP_IN * sizeof(float));
    H2D(w.p, params, IC_MLP_NPARAM * sizeof(float));
    H2D(yall.p, y, n);
    (void)hipMemset(m1.p, 0, IC_MLP_NPARAM * sizeof(float));
    (void)hipMemset(m2.p, 0, IC_MLP_NPARAM * sizeof(float));
    hipLaunchKernelGGL(k_normalise, dim3(((long)n * IC_MLP_IN + 255) / 256), dim3(256), 0, s, rawd.p, mean.p, istd.p,
                       n, xall.p);
    hipLaunchKernelGGL(k_to_bf16, dim3((IC_MLP_NPARAM + 255) / 256), dim3(256), 0, s, w.p, wb.p, (long)IC_MLP_NPARAM);
    // deterministic shuffle per epoch (xorshift on the host), rows gathered by copies
    std::vector<long> order(n);
    for (long b = 0; b < n; ++b) order[b] = b;
    uint64_t st = hp.seed * 2654435761ull + 88172645463325252ull;
    auto rnd = [&]() {
        st ^= st << 13;
        st ^= st >> 7;
        st ^= st << 17;
        return st;
    };
    long t = 0;
    std::vector<double> lsums(std::max(nbatch, 1L));
    for (int ep = 0; ep < hp.epochs; ++ep) {
        for (long b = n - 1; b > 0; --b) std::swap(order[b], order[rnd() % (uint64_t)(b + 1)]);
        H2D(orderd.p, order.data(), n * sizeof(long));
        long q = 0;
        for (long b0 = 0; b0 + B <= n; b0 += B, ++q) {
            hipLaunchKernelGGL(k_gather, dim3(((long)B * IC_MLP_IN + 255) / 256), dim3(256), 0, s, xall.p, yall.p,
                               orderd.p, b0, B, xb.p, yb.p);
            fwd_bwd(s, B, xb.p, yb.p, pw, w.p, wb.p, grad.p, loss.p, H1, H2, dz, dZ2, dZ2b, dH1, dZ1, dZ1b, work.p);
            hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, s, (const float *)loss.p, B, lossacc.p, q);
            ++t;
            const float c1 = 1.f - std::pow(hp.beta1, (float)t), c2 = 1.f - std::pow(hp.beta2, (float)t);
            hipLaunchKernelGGL(k_adam, dim3((IC_MLP_NPARAM + 255) / 256), dim3(256), 0, s, w.p, wb.p, grad.p, m1.p,
                               m2.p, IC_MLP_NPARAM, hp.lr, hp.beta1, hp.beta2, hp.eps, c1, c2);
        }
        // the epoch's minibatch losses, summed in batch order
        if (q > 0 && hipMemcpy(lsums.data(), lossacc.p, q * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
            throw std::runtime_error("hipMemcpy failed");
        double lsum = 0.0;
        for (long i = 0; i < q; ++i) lsum += lsums[i];
        if (loss_epochs) loss_epochs[ep] = q ? (float)(lsum / (double)(q * B)) : 0.f;
    }
    if (hipMemcpy(params, w.p, IC_MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        throw std::runtime_error("hipMemcpy failed");
    std::memcpy(mean_out, mean_h.data(), IC_MLP_IN * sizeof(float));
    std::memcpy(std_out, std_h.data(), IC_MLP_IN * sizeof(float));
}

void mlp_infer(const float *raw, long n, const float *params, const float *mean, const float *std, float *prob)
{
    MlpDevice d;
    d.set(params, mean, std);
    const long chunk = 65536;
    d.reserve((int)std::min(n, chunk));
    Buf<float> rawd((size_t)std::min(n, chunk) * IC_MLP_IN);
    for (long b0 = 0; b0 < n; b0 += chunk) {
        const long m = std::min(chunk, n - b0);
        if (hipMemcpy(rawd.p, raw + b0 * IC_MLP_IN, (size_t)m * IC_MLP_IN * sizeof(float), hipMemcpyHostToDevice) !=
            hipSuccess)
            throw std::runtime_error("hipMemcpy failed");
        hipLaunchKernelGGL(k_normalise, dim3((m * IC_MLP_IN + 255) / 256), dim3(256), 0, 0, rawd.p, d.mean, d.istd, m,
                           d.xb);
        d.forward(0, (int)m);
        if (hipMemcpy(prob + b0, d.prob, m * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
            throw std::runtime_error("hipMemcpy failed");
    }
}

// ---------------------------------------------------------------------------
// inference without allocation
// ---------------------------------------------------------------------------
// The scratch of the allocation-free entry point: bf16 weights, 1/std, and
// the bf16 inputs and both hidden layers of up to IC_MLP_NOALLOC_ROWS rows
// (6.2 MiB), one copy per device for the life of the process.  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name is a host-side stand-in).
namespace {
constexpr size_t na_align(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kNaWb = 0;
constexpr size_t kNaIstd = kNaWb + na_align((size_t)IC_MLP_NPARAM * sizeof(uint16_t));
constexpr size_t kNaX = kNaIstd + na_align((size_t)IC_MLP_IN * sizeof(float));
constexpr size_t kNaH1 = kNaX + (size_t)IC_MLP_NOALLOC_ROWS * IC_MLP_IN * sizeof(uint16_t);
constexpr size_t kNaH2 = kNaH1 + (size_t)IC_MLP_NOALLOC_ROWS * IC_MLP_HID * sizeof(uint16_t);
constexpr size_t kNaBytes = kNaH2 + (size_t)IC_MLP_NOALLOC_ROWS * IC_MLP_HID * sizeof(uint16_t);
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {
constexpr int kNaMaxDevices = 64;
unsigned char *g_na_scratch[kNaMaxDevices];   // device address of each device's copy, once resolved
std::mutex g_na_mu;

// Device address of the current device's scratch, resolved on the first call
// on that device.
unsigned char *noalloc_scratch()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) throw std::runtime_error("hipGetDevice failed");
    if (dev < 0 || dev >= kNaMaxDevices) throw std::runtime_error("device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw std::runtime_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_na_scratch[dev] = (unsigned char *)p;
    }
    return g_na_scratch[dev];
}
}  // namespace

void mlp_infer_noalloc(const float *raw, long n, const float *params, const float *mean, const float *std,
                       float *prob, hipStream_t s)
{
    if (n < 0 || n > IC_MLP_NOALLOC_ROWS) throw std::invalid_argument("row count outside 0 .. IC_MLP_NOALLOC_ROWS");
    unsigned char *base = noalloc_scratch();
    if (n == 0) return;
    uint16_t *wb = (uint16_t *)(base + kNaWb);
    float *istd = (float *)(base + kNaIstd);
    uint16_t *xb = (uint16_t *)(base + kNaX);
    uint16_t *h1 = (uint16_t *)(base + kNaH1);
    uint16_t *h2 = (uint16_t *)(base + kNaH2);
    // every scratch element read below is written first in this call: nothing to clear
    hipLaunchKernelGGL(k_istd, dim3((IC_MLP_IN + 255) / 256), dim3(256), 0, s, std, istd);
    hipLaunchKernelGGL(k_to_bf16, dim3((IC_MLP_NPARAM + 255) / 256), dim3(256), 0, s, params, wb, (long)IC_MLP_NPARAM);
    hipLaunchKernelGGL(k_normalise, dim3((n * IC_MLP_IN + 255) / 256), dim3(256), 0, s, raw, mean, istd, n, xb);
    gemm(s, xb, IC_MLP_IN, 1, wb + IC_MLP_OFF_W1, IC_MLP_HID, 1, (int)n, IC_MLP_HID, IC_MLP_IN, params + IC_MLP_OFF_B1,
         1, nullptr, h1, IC_MLP_HID);
    gemm(s, h1, IC_MLP_HID, 1, wb + IC_MLP_OFF_W2, IC_MLP_HID, 1, (int)n, IC_MLP_HID, IC_MLP_HID,
         params + IC_MLP_OFF_B2, 1, nullptr, h2, IC_MLP_HID);
    hipLaunchKernelGGL(k_head, dim3((n + 255) / 256), dim3(256), 0, s, h2, wb + IC_MLP_OFF_W3, params + IC_MLP_OFF_B3,
                       (int)n, (const uint8_t *)nullptr, 0.f, (float *)nullptr, prob, (float *)nullptr,
                       (float *)nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw std::runtime_error(std::string("launch failed: ") + hipGetErrorString(e));
}
