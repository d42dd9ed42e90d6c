// pm_mlp.hip -- surrogate MLP of the forward map: BF16 MFMA forward/backward,
// FP32 Adam (C ABI in include/pm_mlp.h).
//
// GEMM: one 256-thread block computes a 64x64 tile of C = op(A) op(B) with
// 4 waves of 32x32 (2x2 tiles of v_mfma_f32_16x16x32_bf16), stepping K by 32
// through LDS.  Operand fragments (gfx950, 16x16x32 bf16): lane l holds
// A[row l%16][k 8(l/16)..+7] and B[k 8(l/16)..+7][col l%16]; the accumulator
// holds C[rows 4(l/16)..+3][col l%16].  op(A) = A or A^T and op(B) = B or B^T
// cover the forward products H W, the input gradients dZ W^T and the weight
// gradients H^T dZ.  Epilogues fuse bias + GELU (forward) and the GELU
// derivative (backward).  A product whose K exceeds SPLIT_KC is split along K
// (partial products in scratch, added in order by k_split_epilogue, which
// then applies the epilogue), so that the small products of the surrogate
// still spread over the chip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "../../include/pm_mlp.h"
#include "pm_kernels.h"

namespace pm {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_GELU_GRAD = 2 };

struct GemmArgs {
    int M, N, K;
    const bf16 *A;
    int lda;
    const bf16 *B;
    int ldb;
    float *C;  // fp32 result (pre-activation, dZ or plain product)
    int ldc;
    const float *bias;  // EPI_BIAS_GELU / optional for EPI_STORE
    bf16 *H;            // bf16 copy of the activation (or of dZ)
    int ldh;
    const float *Z;  // saved pre-activation for EPI_GELU_GRAD
    int ldz;
    // split K: block z of the grid reduces k in [z kc, (z + 1) kc) into
    // C + z c_split (plain products; gemm() sets these, kc = 0: all of K)
    int kc;
    int64_t c_split;
    float *part;  // scratch for split-K partial products (nullptr: no split)
};

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

constexpr int TM = 64, TN = 64, TK = 32, LDSK = TK + 8;  // padded rows against bank conflicts

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const GemmArgs g)
{
    __shared__ __align__(16) bf16 As[TM][LDSK];
    __shared__ __align__(16) bf16 Bs[TN][LDSK];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int bm = blockIdx.y * TM, bn = blockIdx.x * TN;
    const int kb = g.kc ? (int)blockIdx.z * g.kc : 0;
    const int ke = g.kc ? (kb + g.kc < g.K ? kb + g.kc : g.K) : g.K;
    float *const C = g.C + (int64_t)blockIdx.z * g.c_split;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16 zero = (bf16)0.0f;

    // 16-byte loads (8 bf16 along the contiguous dimension, one per thread
    // per operand tile) where a whole tile is in range and the rows are
    // 16-byte aligned; element loads otherwise
    const bool a_vec = bm + TM <= g.M && g.lda % 8 == 0 && (reinterpret_cast<uintptr_t>(g.A) & 15) == 0;
    const bool b_vec = bn + TN <= g.N && g.ldb % 8 == 0 && (reinterpret_cast<uintptr_t>(g.B) & 15) == 0;
    for (int k0 = kb; k0 < ke; k0 += TK) {
        const bool full_k = k0 + TK <= ke && k0 % 8 == 0;
        if (a_vec && full_k) {
            if (!TA) {  // A[m][k]: 8 consecutive k of row m -> one LDS row segment
                const int r = tid >> 2, kk = 8 * (tid & 3);
                *reinterpret_cast<uint4 *>(&As[r][kk]) =
                    *reinterpret_cast<const uint4 *>(g.A + (int64_t)(bm + r) * g.lda + k0 + kk);
            } else {  // A[k][m]: 8 consecutive m of row k -> column kk of 8 LDS rows
                const int kk = tid >> 3, r = 8 * (tid & 7);
                const uint4 v = *reinterpret_cast<const uint4 *>(g.A + (int64_t)(k0 + kk) * g.lda + bm + r);
                const bf16 *h = reinterpret_cast<const bf16 *>(&v);
#pragma unroll
                for (int i = 0; i < 8; ++i) As[r + i][kk] = h[i];
            }
        } else {
            // op(A)(m, k) -> As[m][k]; the fastest-varying thread index
            // follows the contiguous global dimension.
            for (int e = tid; e < TM * TK; e += 256) {
                int r, kk;
                if (!TA) { r = e / TK; kk = e % TK; }
                else { kk = e / TM; r = e % TM; }
                const int m = bm + r, k = k0 + kk;
                bf16 v = zero;
                if (m < g.M && k < ke) v = TA ? g.A[(int64_t)k * g.lda + m] : g.A[(int64_t)m * g.lda + k];
                As[r][kk] = v;
            }
        }
        if (b_vec && full_k) {
            if (TB) {  // B[n][k]: 8 consecutive k of row n -> one LDS row segment
                const int c = tid >> 2, kk = 8 * (tid & 3);
                *reinterpret_cast<uint4 *>(&Bs[c][kk]) =
                    *reinterpret_cast<const uint4 *>(g.B + (int64_t)(bn + c) * g.ldb + k0 + kk);
            } else {  // B[k][n]: 8 consecutive n of row k -> column kk of 8 LDS rows
                const int kk = tid >> 3, c = 8 * (tid & 7);
                const uint4 v = *reinterpret_cast<const uint4 *>(g.B + (int64_t)(k0 + kk) * g.ldb + bn + c);
                const bf16 *h = reinterpret_cast<const bf16 *>(&v);
#pragma unroll
                for (int i = 0; i < 8; ++i) Bs[c + i][kk] = h[i];
            }
        } else {
            // op(B)(k, n) -> Bs[n][k]
            for (int e = tid; e < TN * TK; e += 256) {
                int c, kk;
                if (!TB) { kk = e / TN; c = e % TN; }
                else { c = e / TK; kk = e % TK; }
                const int n = bn + c, k = k0 + kk;
                bf16 v = zero;
                if (n < g.N && k < ke) v = TB ? g.B[(int64_t)n * g.ldb + k] : g.B[(int64_t)k * g.ldb + n];
                Bs[c][kk] = v;
            }
        }
        __syncthreads();
        const int fr = lane & 15, fk = 8 * (lane >> 4);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&As[wm + 16 * a + fr][fk]);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&Bs[wn + 16 * b + fr][fk]);
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[a][b], 0, 0, 0);
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = bm + wm + 16 * a + 4 * (lane >> 4) + i;
                const int n = bn + wn + 16 * b + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[a][b][i];
                if (EPI == EPI_STORE) {
                    if (g.bias) v += g.bias[n];
                    C[(int64_t)m * g.ldc + n] = v;
                } else if (EPI == EPI_BIAS_GELU) {
                    v += g.bias[n];
                    C[(int64_t)m * g.ldc + n] = v;
                    g.H[(int64_t)m * g.ldh + n] = (bf16)gelu(v);
                } else {
                    v *= gelu_grad(g.Z[(int64_t)m * g.ldz + n]);
                    C[(int64_t)m * g.ldc + n] = v;
                    g.H[(int64_t)m * g.ldh + n] = (bf16)v;
                }
            }
}

// K chunk of split products (a multiple of the K tile).  A product whose K
// exceeds it runs as ceil(K / SPLIT_KC) blocks along z writing plain partial
// products to scratch; k_split_epilogue then adds them in order of z and
// applies the epilogue.  Results do not depend on scheduling.
constexpr int SPLIT_KC = 128;

template <int EPI>
__global__ void k_split_epilogue(const GemmArgs g, int splits)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t count = (int64_t)g.M * g.N;
    if (i >= count) return;
    const int m = (int)(i / g.N), n = (int)(i - (int64_t)m * g.N);
    float v = g.part[i];
    for (int z = 1; z < splits; ++z) v += g.part[(int64_t)z * count + i];
    if (EPI == EPI_STORE) {
        if (g.bias) v += g.bias[n];
        g.C[(int64_t)m * g.ldc + n] = v;
    } else if (EPI == EPI_BIAS_GELU) {
        v += g.bias[n];
        g.C[(int64_t)m * g.ldc + n] = v;
        g.H[(int64_t)m * g.ldh + n] = (bf16)gelu(v);
    } else {
        v *= gelu_grad(g.Z[(int64_t)m * g.ldz + n]);
        g.C[(int64_t)m * g.ldc + n] = v;
        g.H[(int64_t)m * g.ldh + n] = (bf16)v;
    }
}

static int split_count(int K) { return (K + SPLIT_KC - 1) / SPLIT_KC; }

template <bool TA, bool TB, int EPI>
static hipError_t gemm(const GemmArgs &g0, hipStream_t st)
{
    const int splits = g0.part ? split_count(g0.K) : 1;
    if (splits <= 1) {
        GemmArgs g = g0;
        g.kc = 0;
        g.c_split = 0;
        dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM, 1);
        hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, st, g);
        return hipGetLastError();
    }
    GemmArgs p = g0;  // partial products into scratch, M x N each
    p.C = g0.part;
    p.ldc = g0.N;
    p.bias = nullptr;
    p.kc = SPLIT_KC;
    p.c_split = (int64_t)g0.M * g0.N;
    dim3 grid((p.N + TN - 1) / TN, (p.M + TM - 1) / TM, splits);
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI_STORE>), grid, dim3(256), 0, st, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t count = (int64_t)g0.M * g0.N;
    hipLaunchKernelGGL((k_split_epilogue<EPI>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, g0, splits);
    return hipGetLastError();
}

// h0 = bf16(x * in_scale)
__global__ void k_prep_in(const float *__restrict__ x, const float *__restrict__ scale, int n, int d,
                          bf16 *__restrict__ h)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * d) return;
    h[e] = (bf16)(x[e] * scale[e % d]);
}

// y_phys = y * out_std + out_mean
__global__ void k_out_affine(const float *__restrict__ y, const float *__restrict__ mu,
                             const float *__restrict__ sd, int n, int d, float *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * d) return;
    const int j = (int)(e % d);
    out[e] = y[e] * sd[j] + mu[j];
}

// dL/dy of L = 1/(n d) sum (y - (t - mu)/sd)^2, and L itself (atomic sum).
__global__ void k_loss_grad(const float *__restrict__ y, const float *__restrict__ t,
                            const float *__restrict__ mu, const float *__restrict__ sd, int n, int d,
                            float *__restrict__ dy, bf16 *__restrict__ dyb, float *__restrict__ loss)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float contrib = 0.f;
    if (e < (int64_t)n * d) {
        const int j = (int)(e % d);
        const float r = y[e] - (t[e] - mu[j]) / sd[j];
        const float gsc = 2.0f / ((float)n * (float)d);
        dy[e] = gsc * r;
        dyb[e] = (bf16)(gsc * r);
        contrib = r * r / ((float)n * (float)d);
    }
    // wave reduction, one atomic per wave
    for (int off = 32; off >= 1; off >>= 1) contrib += __shfl_xor(contrib, off, 64);
    if ((threadIdx.x & 63) == 0 && loss) atomicAdd(loss, contrib);
}

// db[j] = sum_m dz[m][j] in two passes.  k_colsum: block (x, r) takes 64
// columns and rows r, r + CS_CHUNKS, ...; thread (g, c) of its 1024 sums
// every CS_GROUPS-th of those rows of column c (coalesced rows of 64 floats
// per wave) and the 16 row groups are added in a fixed order through LDS into
// part[r][j].  k_colsum_rows adds the CS_CHUNKS partial rows in order.  The
// result does not depend on scheduling.
constexpr int CS_COLS = 64, CS_GROUPS = 16, CS_CHUNKS = 16;
__global__ __launch_bounds__(1024) void k_colsum(const float *__restrict__ dz, int n, int d,
                                                 float *__restrict__ part)
{
    __shared__ float acc[CS_GROUPS][CS_COLS];
    const int c = threadIdx.x & (CS_COLS - 1), g = threadIdx.x / CS_COLS;
    const int j = blockIdx.x * CS_COLS + c, r = blockIdx.y;
    float s0 = 0.f, s1 = 0.f;
    if (j < d) {
        int m = r + CS_CHUNKS * g;
        for (; m + CS_CHUNKS * CS_GROUPS < n; m += 2 * CS_CHUNKS * CS_GROUPS) {
            s0 += dz[(int64_t)m * d + j];
            s1 += dz[(int64_t)(m + CS_CHUNKS * CS_GROUPS) * d + j];
        }
        if (m < n) s0 += dz[(int64_t)m * d + j];
    }
    acc[g][c] = s0 + s1;
    __syncthreads();
    if (g == 0 && j < d) {
        float t = 0.f;
        for (int q = 0; q < CS_GROUPS; ++q) t += acc[q][c];
        part[(int64_t)r * d + j] = t;
    }
}

__global__ void k_colsum_rows(const float *__restrict__ part, int d, float *__restrict__ db)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d) return;
    float t = 0.f;
    for (int r = 0; r < CS_CHUNKS; ++r) t += part[(int64_t)r * d + j];
    db[j] = t;
}

__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, bf16 *__restrict__ ws, int64_t P, float lr, float c1, float c2)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P) return;
    const float gi = g[e];
    const float a = 0.9f * m1[e] + 0.1f * gi;
    const float b = 0.999f * m2[e] + 0.001f * gi * gi;
    m1[e] = a;
    m2[e] = b;
    const float wi = w[e] - lr * (a * c1) / (sqrtf(b * c2) + 1e-8f);
    w[e] = wi;
    ws[e] = (bf16)wi;
}

__global__ void k_to_bf16(const float *__restrict__ w, bf16 *__restrict__ ws, int64_t P)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < P) ws[e] = (bf16)w[e];
}

__global__ void k_zero_f32(float *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

static dim3 g1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace pm

using namespace pm;

struct pm_mlp {
    pm_ctx *ctx = nullptr;
    int d_in = 0, h = 0, L = 0, d_out = 0, max_batch = 0;
    int64_t P = 0;
    std::vector<int> Kd, Nd;            // per linear layer (L + 1 of them)
    std::vector<int64_t> offW, offB;    // offsets in the flat parameter vector
    float *w = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
    bf16 *ws = nullptr;                 // bf16 shadow of w (same offsets)
    float *in_scale = nullptr, *out_mean = nullptr, *out_std = nullptr;
    std::vector<bf16 *> H;              // H[0..L] activations (bf16)
    std::vector<float *> Z;             // Z[1..L] pre-activations (fp32)
    float *Y = nullptr, *dY = nullptr, *loss = nullptr;
    bf16 *dYb = nullptr;
    float *dZ[2] = {nullptr, nullptr};
    bf16 *dZb[2] = {nullptr, nullptr};
    float *part = nullptr;  // split-K partial weight gradients
    int64_t step = 0;
    std::vector<void *> allocs;
};

namespace {

int mlp_alloc(pm_mlp *m, void **p, size_t bytes)
{
    if (hipMalloc(p, bytes ? bytes : 16) != hipSuccess) {
        *p = nullptr;
        return PM_ENOMEM;
    }
    m->allocs.push_back(*p);
    return PM_OK;
}

void mlp_free(pm_mlp *m)
{
    for (void *p : m->allocs) (void)hipFree(p);
    m->allocs.clear();
}

bool mlp_ok(const pm_mlp *m) { return m && !ctx_closed(m->ctx); }

int forward_impl(pm_mlp *m, const float *x, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_prep_in, g1((int64_t)n * m->d_in), dim3(256), 0, st, x, m->in_scale, n, m->d_in, m->H[0]);
    for (int l = 0; l <= m->L; ++l) {
        GemmArgs a{};
        a.M = n;
        a.N = m->Nd[l];
        a.K = m->Kd[l];
        a.A = m->H[l];
        a.lda = m->Kd[l];
        a.B = m->ws + m->offW[l];
        a.ldb = m->Nd[l];
        a.bias = m->w + m->offB[l];
        a.part = m->part;
        if (l < m->L) {
            a.C = m->Z[l + 1];
            a.ldc = m->h;
            a.H = m->H[l + 1];
            a.ldh = m->h;
            if (gemm<false, false, EPI_BIAS_GELU>(a, st) != hipSuccess) return PM_EDEVICE;
        } else {
            a.C = m->Y;
            a.ldc = m->d_out;
            if (gemm<false, false, EPI_STORE>(a, st) != hipSuccess) return PM_EDEVICE;
        }
    }
    return PM_OK;
}

// forward + loss + backward into m->g (logical layout)
int grads_impl(pm_mlp *m, const float *x, const float *t, int n, float *loss, hipStream_t st)
{
    int s = forward_impl(m, x, n, st);
    if (s) return s;
    if (loss) hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, st, loss, 1);
    hipLaunchKernelGGL(k_loss_grad, g1((int64_t)n * m->d_out), dim3(256), 0, st, m->Y, t, m->out_mean, m->out_std, n,
                       m->d_out, m->dY, m->dYb, loss);
    // output layer
    const float *dz = m->dY;
    const bf16 *dzb = m->dYb;
    int cur = 0;
    for (int l = m->L; l >= 0; --l) {
        const int K = m->Kd[l], N = m->Nd[l];
        // dW_l = H_l^T dZ  (K x N, reduction over the batch)
        GemmArgs a{};
        a.M = K;
        a.N = N;
        a.K = n;
        a.A = m->H[l];
        a.lda = K;
        a.B = dzb;
        a.ldb = N;
        a.ldc = N;
        a.C = m->g + m->offW[l];
        a.part = m->part;
        if (gemm<true, false, EPI_STORE>(a, st) != hipSuccess) return PM_EDEVICE;
        hipLaunchKernelGGL(k_colsum, dim3((N + CS_COLS - 1) / CS_COLS, CS_CHUNKS), dim3(CS_COLS * CS_GROUPS), 0, st,
                           dz, n, N, m->part);
        hipLaunchKernelGGL(k_colsum_rows, g1(N), dim3(256), 0, st, m->part, N, m->g + m->offB[l]);
        if (l == 0) break;
        // dZ_{l} (input side) = (dZ W_l^T) * GELU'(Z_l)
        GemmArgs b{};
        b.M = n;
        b.N = K;
        b.K = N;
        b.A = dzb;
        b.lda = N;
        b.B = m->ws + m->offW[l];
        b.ldb = N;
        b.C = m->dZ[cur];
        b.ldc = K;
        b.H = m->dZb[cur];
        b.ldh = K;
        b.Z = m->Z[l];
        b.ldz = K;
        b.part = m->part;
        if (gemm<false, true, EPI_GELU_GRAD>(b, st) != hipSuccess) return PM_EDEVICE;
        dz = m->dZ[cur];
        dzb = m->dZb[cur];
        cur ^= 1;
    }
    return hipGetLastError() == hipSuccess ? PM_OK : PM_EDEVICE;
}

}  // namespace

extern "C" {

int pm_mlp_create(pm_ctx *ctx, int d_in, int d_hidden, int n_hidden, int d_out, int max_batch, uint64_t seed,
                  pm_mlp **out)
{
    if (!out) return PM_EINVAL;
    *out = nullptr;
    if (!ctx || ctx_closed(ctx)) return PM_EINVAL;
    if (d_in < 1 || d_hidden < 1 || n_hidden < 1 || d_out < 1 || max_batch < 1) return PM_EINVAL;
    if (d_in > 65536 || d_hidden > 65536 || d_out > 65536 || n_hidden > 64 || max_batch > (1 << 22))
        return PM_EINVAL;
    if (hipSetDevice(ctx_device(ctx)) != hipSuccess) return PM_EDEVICE;
    pm_mlp *m = new (std::nothrow) pm_mlp();
    if (!m) return PM_ENOMEM;
    m->ctx = ctx;
    m->d_in = d_in;
    m->h = d_hidden;
    m->L = n_hidden;
    m->d_out = d_out;
    m->max_batch = max_batch;
    int64_t off = 0;
    for (int l = 0; l <= n_hidden; ++l) {
        const int K = l == 0 ? d_in : d_hidden;
        const int N = l == n_hidden ? d_out : d_hidden;
        m->Kd.push_back(K);
        m->Nd.push_back(N);
        m->offW.push_back(off);
        off += (int64_t)K * N;
        m->offB.push_back(off);
        off += N;
    }
    m->P = off;
    int st = PM_OK;
    auto A = [&](void **p, size_t bytes) {
        if (st == PM_OK) st = mlp_alloc(m, p, bytes);
    };
    A((void **)&m->w, m->P * 4);
    A((void **)&m->g, m->P * 4);
    A((void **)&m->m1, m->P * 4);
    A((void **)&m->m2, m->P * 4);
    A((void **)&m->ws, m->P * 2);
    A((void **)&m->in_scale, d_in * 4);
    A((void **)&m->out_mean, d_out * 4);
    A((void **)&m->out_std, d_out * 4);
    m->H.assign(n_hidden + 1, nullptr);
    m->Z.assign(n_hidden + 1, nullptr);
    A((void **)&m->H[0], (size_t)max_batch * d_in * 2);
    for (int l = 1; l <= n_hidden; ++l) {
        A((void **)&m->H[l], (size_t)max_batch * d_hidden * 2);
        A((void **)&m->Z[l], (size_t)max_batch * d_hidden * 4);
    }
    A((void **)&m->Y, (size_t)max_batch * d_out * 4);
    A((void **)&m->dY, (size_t)max_batch * d_out * 4);
    A((void **)&m->dYb, (size_t)max_batch * d_out * 2);
    A((void **)&m->loss, 64);
    const int wmax = d_hidden > d_in ? d_hidden : d_in;
    for (int i = 0; i < 2; ++i) {
        A((void **)&m->dZ[i], (size_t)max_batch * wmax * 4);
        A((void **)&m->dZb[i], (size_t)max_batch * wmax * 2);
    }
    {
        // split-K scratch: the largest splits x M x N over the products of a
        // training step (forward H W, weight gradients H^T dZ, input
        // gradients dZ W^T)
        int64_t need = 1;
        for (int l = 0; l <= n_hidden; ++l) {
            const int64_t k = l == 0 ? d_in : d_hidden, nn = l == n_hidden ? d_out : d_hidden;
            need = std::max<int64_t>(need, split_count((int)k) * (int64_t)max_batch * nn);
            need = std::max<int64_t>(need, split_count(max_batch) * k * nn);
            if (l > 0) need = std::max<int64_t>(need, split_count((int)nn) * (int64_t)max_batch * k);
        }
        need = std::max<int64_t>(need, (int64_t)CS_CHUNKS * std::max(d_hidden, d_out));  // column sums
        A((void **)&m->part, (size_t)need * 4);
    }
    if (st) {
        mlp_free(m);
        delete m;
        return st;
    }
    // He-style init N(0, 1/fan_in), zero biases (host RNG, seeded)
    std::vector<float> w(m->P, 0.f);
    std::mt19937_64 rng(seed);
    for (int l = 0; l <= n_hidden; ++l) {
        std::normal_distribution<double> nd(0.0, 1.0 / std::sqrt((double)m->Kd[l]));
        for (int64_t e = 0; e < (int64_t)m->Kd[l] * m->Nd[l]; ++e) w[m->offW[l] + e] = (float)nd(rng);
    }
    std::vector<float> ones(d_in > d_out ? d_in : d_out, 1.f), zeros(d_out, 0.f);
    ctx_retain(ctx);
    *out = m;
    if ((st = pm_mlp_set_params(m, w.data())) || (st = pm_mlp_set_io(m, ones.data(), zeros.data(), ones.data()))) {
        pm_mlp_destroy(m);
        *out = nullptr;
        return st;
    }
    return PM_OK;
}

void pm_mlp_destroy(pm_mlp *m)
{
    if (!m) return;
    (void)hipSetDevice(ctx_device(m->ctx));
    if (!ctx_closed(m->ctx)) (void)hipStreamSynchronize(ctx_stream(m->ctx));
    else (void)hipDeviceSynchronize();
    mlp_free(m);
    ctx_drop(m->ctx);
    delete m;
}

int64_t pm_mlp_n_params(const pm_mlp *m) { return m ? m->P : 0; }

int pm_mlp_set_params(pm_mlp *m, const float *host)
{
    if (!mlp_ok(m) || !host) return PM_EINVAL;
    if (hipSetDevice(ctx_device(m->ctx)) != hipSuccess) return PM_EDEVICE;
    hipStream_t st = ctx_stream(m->ctx);
    if (hipStreamSynchronize(st) != hipSuccess) return PM_EDEVICE;
    if (hipMemcpy(m->w, host, m->P * 4, hipMemcpyHostToDevice) != hipSuccess) return PM_EDEVICE;
    if (hipMemset(m->m1, 0, m->P * 4) != hipSuccess || hipMemset(m->m2, 0, m->P * 4) != hipSuccess) return PM_EDEVICE;
    hipLaunchKernelGGL(k_to_bf16, g1(m->P), dim3(256), 0, st, m->w, m->ws, m->P);
    m->step = 0;
    return hipStreamSynchronize(st) == hipSuccess ? PM_OK : PM_EDEVICE;
}

int pm_mlp_get_params(pm_mlp *m, float *host)
{
    if (!mlp_ok(m) || !host) return PM_EINVAL;
    if (hipSetDevice(ctx_device(m->ctx)) != hipSuccess) return PM_EDEVICE;
    if (hipStreamSynchronize(ctx_stream(m->ctx)) != hipSuccess) return PM_EDEVICE;
    return hipMemcpy(host, m->w, m->P * 4, hipMemcpyDeviceToHost) == hipSuccess ? PM_OK : PM_EDEVICE;
}

int pm_mlp_set_io(pm_mlp *m, const float *in_scale, const float *out_mean, const float *out_std)
{
    if (!mlp_ok(m)) return PM_EINVAL;
    if (out_std)
        for (int j = 0; j < m->d_out; ++j)
            if (!(out_std[j] > 0.f) || !std::isfinite(out_std[j])) return PM_EINVAL;
    if (hipSetDevice(ctx_device(m->ctx)) != hipSuccess) return PM_EDEVICE;
    if (hipStreamSynchronize(ctx_stream(m->ctx)) != hipSuccess) return PM_EDEVICE;
    if (in_scale && hipMemcpy(m->in_scale, in_scale, m->d_in * 4, hipMemcpyHostToDevice) != hipSuccess) return PM_EDEVICE;
    if (out_mean && hipMemcpy(m->out_mean, out_mean, m->d_out * 4, hipMemcpyHostToDevice) != hipSuccess) return PM_EDEVICE;
    if (out_std && hipMemcpy(m->out_std, out_std, m->d_out * 4, hipMemcpyHostToDevice) != hipSuccess) return PM_EDEVICE;
    return PM_OK;
}

int pm_mlp_forward(pm_mlp *m, const float *x, int n, float *y)
{
    if (!mlp_ok(m) || !x || !y || n < 1 || n > m->max_batch) return PM_EINVAL;
    if (hipSetDevice(ctx_device(m->ctx)) != hipSuccess) return PM_EDEVICE;
    hipStream_t st = ctx_stream(m->ctx);
    int s = forward_impl(m, x, n, st);
    if (s) return s;
    hipLaunchKernelGGL(k_out_affine, g1((int64_t)n * m->d_out), dim3(256), 0, st, m->Y, m->out_mean, m->out_std, n,
                       m->d_out, y);
    return hipGetLastError() == hipSuccess ? PM_OK : PM_EDEVICE;
}

int pm_mlp_train_step(pm_mlp *m, const float *x, const float *t, int n, float lr, float *loss)
{
    if (!mlp_ok(m) || !x || !t || n < 1 || n > m->max_batch || !(lr > 0.f) || !std::isfinite(lr)) return PM_EINVAL;
    if (hipSetDevice(ctx_device(m->ctx)) != hipSuccess) return PM_EDEVICE;
    hipStream_t st = ctx_stream(m->ctx);
    int s = grads_impl(m, x, t, n, loss, st);
    if (s) return s;
    m->step += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)m->step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)m->step)));
    hipLaunchKernelGGL(k_adam, g1(m->P), dim3(256), 0, st, m->w, m->g, m->m1, m->m2, m->ws, m->P, lr, c1, c2);
    return hipGetLastError() == hipSuccess ? PM_OK : PM_EDEVICE;
}

int pm_mlp_grads(pm_mlp *m, const float *x, const float *t, int n, float *host_grads)
{
    if (!mlp_ok(m) || !x || !t || !host_grads || n < 1 || n > m->max_batch) return PM_EINVAL;
    if (hipSetDevice(ctx_device(m->ctx)) != hipSuccess) return PM_EDEVICE;
    hipStream_t st = ctx_stream(m->ctx);
    int s = grads_impl(m, x, t, n, m->loss, st);
    if (s) return s;
    if (hipStreamSynchronize(st) != hipSuccess) return PM_EDEVICE;
    return hipMemcpy(host_grads, m->g, m->P * 4, hipMemcpyDeviceToHost) == hipSuccess ? PM_OK : PM_EDEVICE;
}

}  // extern "C"
