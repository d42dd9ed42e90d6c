// pm_mx.hip -- the velocity field of eq. v_expand on the torus for small
// wavenumber cutoffs (1 <= K <= 8; basis entries 0..15 of each axis on the
// matrix cores, the entry-16 terms of K = 8 on the vector units), FP32
// particles; the same for the disk's three forms (K <= 4) inside the walk of
// Algorithm 2.
//
// With the axis bases phi_0 = 1, phi_{2n-1} = cos 2 pi n s, phi_{2n} =
// sin 2 pi n s the field is
//     v_x(x, y) = phi(x)^T Cx phi(y),   v_y(x, y) = phi(x)^T Cy phi(y),
// 2 B^2 multiply-adds per particle (338 at K = 6), about three quarters of
// all the arithmetic of an Euler-Maruyama step.  For the 64 particles of a
// wave the inner products W = [Cx; Cy]^T Phi_x are one dense contraction
// (32 rows: 16 per component, B <= 16 x-basis functions, 64 particles) on
// v_mfma_f32_32x32x16_f16.  Operands are split into FP16 pairs (a = a_hi +
// a_lo) and three products a_hi b_hi + a_hi b_lo + a_lo b_hi are accumulated
// in FP32: about 2^-22 relative error per product.  The coefficients enter
// scaled by a power of two that puts max |C| in [2^14, 2^15), so their low
// halves stay normal FP16 numbers, and the result is scaled back exactly.
// The x basis enters unscaled: the low halves of entries below 2^-3 are FP16
// subnormals, which the matrix cores take exactly (an in-bounds product of
// subnormal operands on gfx950 equals the exact sum), so such an entry keeps
// an absolute resolution of 2^-25, below the relative error of the split
// products.
//
// Matrix-core layouts (32x32x16, lane l, h = l / 32):
//   A (32 rows x 16 cols i): lane l holds row l % 32, cols i = 8 h + e (e = 0..7);
//                            row q < 16 is Cx[i][j = q], row q >= 16 is Cy[i][j = q - 16]
//   B (16 rows i x 32 cols): lane l holds phi_{8 h + e}(x_p), p = 32 b + l % 32 (column block b)
//   D (32 x 32, FP32):       lane l holds W[q = 8 (r / 4) + 4 h + r % 4][p = 32 b + l % 32], r = 0..15
// Lane l holds particle l.  Every lane computes its own particle's bases; one
// v_permlane32_swap per register pair (it swaps the upper half-wave of one
// register with the lower half-wave of another) moves the halves that the
// other half-wave's lanes need: lanes l and l ^ 32 exchange x-basis entries
// 8..15 / 0..7, and y-basis entries {4..7, 12..15} / {0..3, 8..11}, the rows
// that their D registers hold.  A last swap pairs the two half sums of each
// particle in a fixed order, so the result is identical in every launch
// shape.
#include "pm_mx.h"
#include "pm_split.h"
#include "pm_walk.h"

namespace pm {

typedef _Float16 h16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Operand packing: FP64 coefficients (torus rows of k_fold: row j holds
// Cx[i][j], Cy[i][j] at [2i], [2i+1]) -> scaled FP16 pairs in the A layout.
// One block per parameter set; a fixed max-reduction tree.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pack_mx(const MxPackArgs a, unsigned char *__restrict__ out)
{
    __shared__ double red[256];
    const int B = 2 * a.K + 1;
    const int R = a.row_stride;
    const int nf = a.domain == PM_DISK ? 3 : 2;  // forms per row: (Psi,) Cx, Cy
    const double *__restrict__ C = a.coef + (int64_t)blockIdx.x * a.coef_stride;
    double m = 0.0;
    for (int e = threadIdx.x; e < nf * B * B; e += blockDim.x) {
        const int j = e / (nf * B), q = e % (nf * B);
        m = fmax(m, fabs(C[j * R + q]));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const double cmax = red[0];
    // velocity bound: the larger of sum |Cx| and sum |Cy| over the whole
    // matrix (every basis function is bounded by 1); torus only
    double vb = 0.0;
    if (nf == 2) {
        double sx = 0.0, sy = 0.0;
        for (int e = threadIdx.x; e < B * B; e += blockDim.x) {
            const int j = e / B, i = e % B;
            sx += fabs(C[j * R + 2 * i]);
            sy += fabs(C[j * R + 2 * i + 1]);
        }
        __syncthreads();
        red[threadIdx.x] = fmax(sx, sy);
        __syncthreads();
        // sum of the per-thread maxima >= max of the two sums
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        vb = red[0];
    }
    int sc = 0;
    if (cmax > 0.0) {
        int ex;
        frexp(cmax, &ex);  // cmax = f 2^ex, f in [0.5, 1)
        sc = 15 - ex;
        // tiny fields keep a representable scale (their velocity is ~0 anyway)
        sc = sc > 100 ? 100 : (sc < -100 ? -100 : sc);
    }
    unsigned char *set = out + (int64_t)blockIdx.x * MX_SET_BYTES;
    MxHeader *hd = reinterpret_cast<MxHeader *>(set);
    if (threadIdx.x == 0) {
        hd->inv_scale = ldexpf(1.f, -(sc + MX_BASIS_SHIFT));
        hd->scale = ldexpf(1.f, sc + MX_BASIS_SHIFT);
        hd->cmax = (float)cmax;
        hd->vbound = (float)(vb * (1.0 + 0x1p-10));  // covers FP32 rounding of the bound and the bases
        for (int q = 0; q < 12; ++q) hd->pad[q] = 0.f;
    }
    _Float16 *hi = reinterpret_cast<_Float16 *>(set + sizeof(MxHeader));
    _Float16 *lo = hi + 64 * 8;
    for (int t = threadIdx.x; t < 64 * 8; t += blockDim.x) {
        const int lane = t >> 3, e = t & 7;
        const int row = lane & 31, i = mx_x_entry(a.K, 8 * (lane >> 5) + e);
        int comp, j;
        if (nf == 2) {  // torus: rows 0..15 Cx, 16..31 Cy; row 8(q/4) + 4h + q%4 is register q, half h
            comp = row >> 4;
            const int r = row & 15;
            j = mx_y_entry(a.K, 4 * (r >> 3) + (r & 3), (r >> 2) & 1);
        } else {  // disk: rows 8f + j (j < 8) and 24 + f (j = 8) for form f
            comp = row < 24 ? row >> 3 : (row < 27 ? row - 24 : -1);
            j = row < 24 ? row & 7 : 8;
        }
        double v = 0.0;
        if (comp >= 0 && i >= 0 && i < B && j >= 0 && j < B) v = ldexp(C[j * R + nf * i + comp], sc);
        const _Float16 h = (_Float16)(float)v;
        hi[t] = h;
        lo[t] = (_Float16)(float)(v - (double)(float)h);
    }
    // K = 8 (torus): the entry-16 row and column, FP32, unscaled (the column
    // carries 2^-8 against the x basis' scale); zeros otherwise
    float *border = reinterpret_cast<float *>(set + MX_BORDER_OFFSET);
    for (int t = threadIdx.x; t < MX_BORDER_FLOATS + 2; t += blockDim.x) {
        float v = 0.f;
        if (nf == 2 && B == 17 && t < MX_BORDER_FLOATS) {
            if (t < 34) {
                const int c = t / 17, j = t % 17;  // C_c[16][j]
                v = (float)C[j * R + 2 * 16 + c];
            } else {
                const int c = (t - 34) / 16, i = (t - 34) % 16;  // C_c[i][16]
                v = (float)ldexp(C[16 * R + 2 * i + c], -MX_BASIS_SHIFT);
            }
        }
        border[t] = v;
    }
}

// ---------------------------------------------------------------------------
// Velocity of the 64 particles of a wave at (xh, yh); every lane of the wave
// must call it (lanes without a particle pass any finite position).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void swap_halves(uint32_t &p, uint32_t &q)
{
    const auto s = __builtin_amdgcn_permlane32_swap(p, q, false, false);
    p = s[0];
    q = s[1];
}

__device__ __forceinline__ void swap_halves(float &p, float &q)
{
    uint32_t a = __builtin_bit_cast(uint32_t, p), b = __builtin_bit_cast(uint32_t, q);
    swap_halves(a, b);
    p = __builtin_bit_cast(float, a);
    q = __builtin_bit_cast(float, b);
}

// phi[0] = S, phi[2n-1] = S cos(2 pi n s), phi[2n] = S sin(2 pi n s) for
// n = 1..K (S = 2^MX_BASIS_SHIFT for the x basis, 1 for the y basis), the
// harmonics n >= 2 by the three-term (Chebyshev) recurrences
//   cos((n+1)t) = 2 cos t cos(nt) - cos((n-1)t),
//   sin((n+1)t) = 2 cos t sin(nt) - sin((n-1)t),
// one FMA per entry.  Scaling by a power of two commutes with every rounding,
// so the x entries are exactly S times the unscaled ones.  In FP32 the entries
// up to n = 8 stay within 2.5e-6 of the exact values (1.4e-6 at n = 6, rms
// 3.4e-7), a few times the angle-addition error and below the error budget of
// the split-FP16 products.
template <int K>
__device__ __forceinline__ void cheb_basis(float s, float S, float *phi)
{
    float s1, c1;
    sincos_rev(s, s1, c1);
    const float t = c1 + c1;
    phi[0] = S;
    phi[1] = c1 * S;
    phi[2] = s1 * S;
#pragma unroll
    for (int n = 2; n <= K; ++n) {
        phi[2 * n - 1] = __builtin_fmaf(t, phi[2 * n - 3], -phi[2 * n - 5 < 0 ? 0 : 2 * n - 5]);
        phi[2 * n] = n == 2 ? t * phi[2] : __builtin_fmaf(t, phi[2 * n - 2], -phi[2 * n - 4]);
    }
}

// Operand registers of the tile's padding rows (x-basis entries 8 + 2d,
// 9 + 2d >= B, whose coefficient columns are zero): any finite FP16 values
// serve there.  A caller that evaluates the velocity repeatedly keeps them
// from one call to the next (initially zero), so the swap that moves the
// partner's entries 2d, 2d + 1 needs no fresh zero register each time.
struct MxPad {
    uint32_t h[4] = {0u, 0u, 0u, 0u}, l[4] = {0u, 0u, 0u, 0u};
    // the constant register of both column blocks (hi: entry 0 in FP16, lo: zero)
    uint32_t ch[2] = {(uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(float)(1 << MX_BASIS_SHIFT)),
                      (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(float)(1 << MX_BASIS_SHIFT))};
    uint32_t cl[2] = {0u, 0u};
};

// The contraction W = A^T Phi_x for the 64 particles of a wave: x basis
// (px, from cheb_basis) split into FP16 pairs in the slots of mx_x_entry (P:
// the lower half-wave's registers, Q: the upper's), the half-wave swaps that
// make P the B operand of column block 0 (particles 0..31) and Q that of
// block 1 (32..63), and the three split products per block.  Per register:
// both halves constant or padding: a constant register, the same in every
// lane and block (padding slots meet zero coefficients, so any finite value
// serves there), no swap; both varying: one swap each for hi and lo; P
// varying and Q padding: P is swapped with the carried padding register of
// `pad` (a swap writes the upper half-wave of P and the lower half-wave of
// its partner, so the carried register's upper half keeps its initial zero
// and its lower half receives the partner's P entries, while P's upper half
// takes finite values of the previous call into padding slots); P constant
// and Q varying (K = 7): the constant is set again before each swap.
template <int K>
__device__ __forceinline__ void mx_contract(const h16x8 ahi, const h16x8 alo, const float *px, f32x16 &d0,
                                            f32x16 &d1, MxPad &pad)
{
    static_assert(K >= 1 && K <= MX_MAX_K, "small-K path");
    // register kinds: 0 padding, 1 the constant entry 0 (with padding), 2 varying
    constexpr auto kind = [](int h, int d) {
        const int e0 = mx_x_entry(K, 8 * h + 2 * d), e1 = mx_x_entry(K, 8 * h + 2 * d + 1);
        if (e0 < 0 && e1 < 0) return 0;
        if (e0 == 0 && e1 < 0) return 1;
        return 2;
    };
    // entry 0 in FP16: S in the low half, the padding slot beside it zero
    const uint32_t chi = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(float)(1 << MX_BASIS_SHIFT));
    uint32_t Ph[4], Pl[4], Qh[4], Ql[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int e0 = mx_x_entry(K, 8 * half + 2 * d), e1 = mx_x_entry(K, 8 * half + 2 * d + 1);
            uint32_t hi = 0u, lo = 0u;
            if (kind(half, d) == 2) split_pair(px[e0 < 0 ? 0 : e0], e1 < 0 ? 0.f : px[e1], hi, lo);
            else if (kind(half, d) == 1) hi = chi;
            (half ? Qh : Ph)[d] = hi;
            (half ? Ql : Pl)[d] = lo;
        }
    }
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int kp = kind(0, d), kq = kind(1, d);
        if (kp != 2 && kq != 2) {  // constant or padding in both halves
            if (kp == 1 || kq == 1) {
                __asm__ volatile("" : "+v"(pad.ch[0]), "+v"(pad.ch[1]), "+v"(pad.cl[0]), "+v"(pad.cl[1]));
                Ph[d] = pad.ch[0];
                Qh[d] = pad.ch[1];
                Pl[d] = pad.cl[0];
                Ql[d] = pad.cl[1];
            } else {
                Qh[d] = Ph[d] = 0u;
                Ql[d] = Pl[d] = 0u;
            }
            continue;
        }
        if (kq == 0) {  // Q padding: swap with the carried register
            Qh[d] = pad.h[d];
            Ql[d] = pad.l[d];
        }
        swap_halves(Ph[d], Qh[d]);
        swap_halves(Pl[d], Ql[d]);
        if (kq == 0) {
            pad.h[d] = Qh[d];
            pad.l[d] = Ql[d];
        }
    }
    const h16x8 b0h = __builtin_bit_cast(h16x8, (u32x4){Ph[0], Ph[1], Ph[2], Ph[3]});
    const h16x8 b0l = __builtin_bit_cast(h16x8, (u32x4){Pl[0], Pl[1], Pl[2], Pl[3]});
    const h16x8 b1h = __builtin_bit_cast(h16x8, (u32x4){Qh[0], Qh[1], Qh[2], Qh[3]});
    const h16x8 b1l = __builtin_bit_cast(h16x8, (u32x4){Ql[0], Ql[1], Ql[2], Ql[3]});
    d0 = f32x16{};
    d1 = f32x16{};
    d0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, b0h, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, b1h, d1, 0, 0, 0);
    d0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, b0l, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, b1l, d1, 0, 0, 0);
    d0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(alo, b0h, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(alo, b1h, d1, 0, 0, 0);
}

// Torus: rows r < 16 hold Cx[.][j], rows r >= 16 Cy[.][j], with tile row
// r mod 16 = 8 (q / 4) + 4 h + q mod 4 holding j = mx_y_entry(K, q, h)
// (k_pack_mx): D register q of a lower-half lane meets y entry 2q + 2 and the
// same register of an upper-half lane entry 2q + 1, so one swap of that pair
// serves both column blocks; register min(K, 7) meets the constant entry 0
// (and padding, or entry 15 at K = 8) and the registers past it hold zero
// rows in both halves and drop out.  At K = 8 the tile
// holds i, j <= 15 and the entry-16 row and column come from
// `border` (MX_BORDER_FLOATS, wave-uniform) on the vector units:
//   v_c += phi_16(x) sum_{j<=16} C_c[16][j] phi_j(y) + phi_16(y) sum_{i<16} C_c[i][16] phi_i(x).
// The sums (sx, sy) are in the units of the packed coefficients, v = s x
// inv_scale; `border` holds the border coefficients in the same units (times
// the header's `scale`).  At K <= 7 the rows of entry 0 (times the constant
// 1) start the y-form accumulators.
template <int K>
__device__ __forceinline__ void mx_velocity_sum(const h16x8 ahi, const h16x8 alo, float xh, float yh, float &sx,
                                                float &sy, MxPad &pad, const float *__restrict__ border = nullptr)
{
    constexpr int B = 2 * K + 1;
    float px[17];
    cheb_basis<K>(xh, (float)(1 << MX_BASIS_SHIFT), px);
#pragma unroll
    for (int e = B; e < 17; ++e) px[e] = 0.f;
    f32x16 d0, d1;
    mx_contract<K>(ahi, alo, px, d0, d1, pad);

    // y basis (FP32, unscaled) while the matrix cores work: Py = entries
    // 2q + 2, Qy = entries 2q + 1; after the swaps Py serves column block 0
    // and Qy block 1, matching D register q (x rows) and 8 + q (y rows).
    // Register M = min(K, 7) meets entry 0 (= 1) in the lower half-wave and
    // zero rows in the upper one at K <= 7, so it starts the sums; at K = 8
    // its upper half meets entry 15, carried over by one more swap.
    constexpr int M = K < 7 ? K : 7;
    constexpr int NQ = K == 8 ? M + 1 : M;  // registers multiplied by a y entry
    float py[17];
    cheb_basis<K>(yh, 1.f, py);
#pragma unroll
    for (int e = B; e < 17; ++e) py[e] = 0.f;
    float Py[M + 1], Qy[M + 1];
#pragma unroll
    for (int q = 0; q < M; ++q) {
        Py[q] = py[2 * q + 2];
        Qy[q] = py[2 * q + 1];
        swap_halves(Py[q], Qy[q]);
    }
    Py[M] = 1.f;
    Qy[M] = K == 8 ? py[15] : 1.f;
    if constexpr (K == 8) swap_halves(Py[M], Qy[M]);
    float ax0 = 0.f, ay0 = 0.f, ax1 = 0.f, ay1 = 0.f;
    if constexpr (K < 8) {
        ax0 = d0[M];
        ay0 = d0[8 + M];
        ax1 = d1[M];
        ay1 = d1[8 + M];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        ax0 = __builtin_fmaf(d0[q], Py[q], ax0);
        ay0 = __builtin_fmaf(d0[8 + q], Py[q], ay0);
        ax1 = __builtin_fmaf(d1[q], Qy[q], ax1);
        ay1 = __builtin_fmaf(d1[8 + q], Qy[q], ay1);
    }
    // lane l < 32 owns particle l of block 0 (its rows and those of lane
    // l + 32); lane l >= 32 owns particle l of block 1.  After the swap every
    // lane adds (lower half-wave rows) + (upper half-wave rows).
    swap_halves(ax0, ax1);
    swap_halves(ay0, ay1);
    sx = ax0 + ax1;
    sy = ay0 + ay1;
    if constexpr (K == 8) {
        float r0 = 0.f, r1 = 0.f, s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int j = 0; j < 17; ++j) {
            r0 = __builtin_fmaf(border[j], py[j], r0);
            r1 = __builtin_fmaf(border[17 + j], py[j], r1);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            s0 = __builtin_fmaf(border[34 + i], px[i], s0);
            s1 = __builtin_fmaf(border[50 + i], px[i], s1);
        }
        const float p16 = px[16] * (1.0f / (float)(1 << MX_BASIS_SHIFT));  // phi_16(x), exact
        sx = __builtin_fmaf(r0, p16, __builtin_fmaf(s0, py[16], sx));
        sy = __builtin_fmaf(r1, p16, __builtin_fmaf(s1, py[16], sy));
    }
}

// The velocity itself (no drift): the sums scaled by inv_scale.
template <int K>
__device__ __forceinline__ void mx_velocity(const h16x8 ahi, const h16x8 alo, float inv, float xh, float yh,
                                            float &vx, float &vy, MxPad &pad,
                                            const float *__restrict__ border = nullptr)
{
    float sx, sy;
    mx_velocity_sum<K>(ahi, alo, xh, yh, sx, sy, pad, border);
    vx = sx * inv;
    vy = sy * inv;
}

// Disk, psi = chi psi_F with chi = (1 - r^2)^2 (K <= 4, B <= 9): rows 8f + j
// hold form f (0: Psi, 1: Cx, 2: Cy) at j = 0..7 and rows 24 + f the forms
// at j = 8.  A lane's D registers r = 0..3, 4..7 and 8..11 are the three
// forms at j = 4h + (r mod 4), and r = 12, 13, 14 the j = 8 rows (lower
// half-wave; the upper half's rows 28..31 are zero rows), so five y-basis
// values per particle, {phi_0..3, phi_8} or {phi_4..7, 0}, serve all three
// forms.  Then v = grad-perp (chi psi_F) by the product rule, as the vector
// engine forms it.
template <int K>
__device__ __forceinline__ void mx_velocity_disk(const h16x8 ahi, const h16x8 alo, float inv, float xh, float yh,
                                                 float &vx, float &vy, MxPad &pad)
{
    constexpr int B = 2 * K + 1;
    static_assert(K >= 1 && B <= 9, "disk rows");
    float px[16];
    cheb_basis<K>(xh, (float)(1 << MX_BASIS_SHIFT), px);
#pragma unroll
    for (int e = B; e < 16; ++e) px[e] = 0.f;
    f32x16 d0, d1;
    mx_contract<K>(ahi, alo, px, d0, d1, pad);
    float py[16];
    cheb_basis<K>(yh, 1.f, py);
#pragma unroll
    for (int e = B; e < 16; ++e) py[e] = 0.f;
    float Py[5], Qy[5];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        Py[q] = py[q];
        Qy[q] = py[4 + q];
    }
    Py[4] = py[8];
    Qy[4] = 0.f;
#pragma unroll
    for (int q = 0; q < 5; ++q) swap_halves(Py[q], Qy[q]);
    float f0[2], fx[2], fy[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const f32x16 &D = b ? d1 : d0;
        const float *Y = b ? Qy : Py;
        float s0 = D[12] * Y[4], sx = D[13] * Y[4], sy = D[14] * Y[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            s0 = __builtin_fmaf(D[r], Y[r], s0);
            sx = __builtin_fmaf(D[4 + r], Y[r], sx);
            sy = __builtin_fmaf(D[8 + r], Y[r], sy);
        }
        f0[b] = s0;
        fx[b] = sx;
        fy[b] = sy;
    }
    swap_halves(f0[0], f0[1]);
    swap_halves(fx[0], fx[1]);
    swap_halves(fy[0], fy[1]);
    const float F0 = (f0[0] + f0[1]) * inv, FX = (fx[0] + fx[1]) * inv, FY = (fy[0] + fy[1]) * inv;
    const float w = 1.f - (xh * xh + yh * yh);
    const float chi = w * w;
    const float g4 = 4.f * w * F0;
    vx = __builtin_fmaf(chi, FX, -(g4 * yh));
    vy = __builtin_fmaf(chi, FY, g4 * xh);
}

// ---------------------------------------------------------------------------
// Torus coordinate as a 32-bit fraction of the period, position = X 2^-32:
// the wrap is the modular overflow of the update.  The increment
// -v dt + sqrt(2 kappa dt) z of eq. (euler) is formed in FP32 in units of
// 2^-32 and added as a whole number of units (2.3e-10 of the period, below
// the FP32 velocity error per step).  The velocity is evaluated at the FP32
// value of the position in [-1/2, 1/2).
// ---------------------------------------------------------------------------
struct FixCoord {
    uint32_t X;
    __device__ __forceinline__ void set(double x)
    {
        const double f = x - floor(x);  // [0, 1); 2^32 wraps to 0 below
        X = (uint32_t)(uint64_t)llrint(f * 4294967296.0);
    }
    __device__ __forceinline__ float at() const { return (float)(int32_t)X * 0x1p-32f; }
    __device__ __forceinline__ double value() const { return (double)(int32_t)X * 0x1p-32; }
    // Add an increment of d units, |d| < 2^31, truncated toward zero: where
    // |d| >= 2^23 the FP32 value is a whole number already, below that the
    // truncation moves the particle by less than 2^-32 of the period.
    __device__ __forceinline__ void add(float d) { X += (uint32_t)(int32_t)d; }
    // The increment of eq. (euler) in units: zs is the noise term
    // sqrt(2 kappa dt) z already in units, dt in hi + lo parts.  Any size,
    // reduced modulo the period first: with |d| held below 2^50 units, t = d
    // 2^-32 and t + 1/2 are exact, q = floor(t + 1/2) is the nearest whole
    // number of periods, and r = d - q 2^32 is exact (d and q 2^32 lie
    // within a factor 2 of each other when q != 0) and in [-2^31, 2^31), an
    // FP32 multiple of 128 units near its ends, so its rounding to a whole
    // unit fits 32 bits.
    __device__ __forceinline__ void advance_wide(float vel, float zs, const StepConsts<float> &c)
    {
        float d = __builtin_fmaf(-c.dtl, vel, zs);
        d = __builtin_fmaf(-c.dth, vel, d);
        d = __builtin_fminf(__builtin_fmaxf(d, -0x1p50f), 0x1p50f);
        const float q = __builtin_floorf(__builtin_fmaf(d, 0x1p-32f, 0.5f));
        const float r = __builtin_fmaf(q, -0x1p32f, d);
        X += (uint32_t)(int32_t)__builtin_rintf(r);
    }
};

// Disk coordinate as a signed 32-bit multiple of 2^-30 (range +-2): the
// increment -v dt + sqrt(2 kappa dt) z of eq. (euler) is formed in FP32 in
// units of 2^-30 as one FMA (the normals come from `normals` already times
// sqrt(2 kappa dt) 2^30; dt 2^30 rounded once to FP32) and added as a whole
// number of units, truncated (9.3e-10, below the FP32 velocity error per
// step).  Each increment is clamped to 1/2, so a walker that starts a step
// inside the unit disk stays inside +-1.5 and the coordinate never wraps;
// only steps that would move a particle by more than half the radius, far
// outside any usable time step, are affected.  The exit test reads the exact
// FP64 value.
struct DiskFix {
    int32_t X;
    float h;  // (float)X 2^-30, kept beside X: the exit test of one step and the bases of the next share it
    static __device__ __forceinline__ void normals(uint32_t wa, uint32_t wb, const StepConsts<float> &c, float &z0,
                                                   float &z1)
    {
        box_muller_r2(wa, wb, c.g2, 0.f, 0.f, z0, z1);
    }
    __device__ __forceinline__ void sync() { h = (float)X * 0x1p-30f; }
    __device__ __forceinline__ void set(double x)
    {
        X = (int32_t)llrint(x * 0x1p30);
        sync();
    }
    __device__ __forceinline__ float at() const { return h; }
    __device__ __forceinline__ double value() const { return (double)X * 0x1p-30; }
    __device__ __forceinline__ void advance(float vel, float zs, const StepConsts<float> &c)
    {
        const float d = __builtin_fmaf(-c.dth, vel, zs);
        X += (int32_t)__builtin_fminf(__builtin_fmaxf(d, -0x1p29f), 0x1p29f);
        sync();
    }
    __device__ __forceinline__ void save(double &a, double &b) const
    {
        a = value();
        b = 0.0;
    }
    __device__ __forceinline__ void load(double a, double) { set(a); }
};

// LDS writes of one wave visible to the same wave's later reads.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void load_set(const unsigned char *__restrict__ set, int lane, h16x8 &ahi, h16x8 &alo,
                                         float &inv)
{
    const h16x8 *t = reinterpret_cast<const h16x8 *>(set + sizeof(MxHeader));
    ahi = t[lane];
    alo = t[64 + lane];
    inv = reinterpret_cast<const MxHeader *>(set)->inv_scale;
}

__device__ __forceinline__ float set_vbound(const unsigned char *__restrict__ set)
{
    return reinterpret_cast<const MxHeader *>(set)->vbound;
}

// ---------------------------------------------------------------------------
// Algorithm 1, persistent: one task is one 64-particle chunk of one parameter
// set, one wave per task; lane l of chunk q of observation j runs particle
// i = 64 q + l (the chunk layout and the Philox streams of the vector time
// kernel, so the payoff and reduction kernels are shared).  Register
// budget: 96 per lane (5 waves per SIMD; K = 6 uses 91 without spills, and a
// budget of 80 for 6 waves per SIMD spilled around the step loop for the same
// time per map).
// ---------------------------------------------------------------------------
template <int K, bool MT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_time_mx(
    const MxTimeArgs m)
{
    // K = 8: the border coefficients of the wave's parameter set, re-read from
    // LDS at every step (broadcast) rather than held in 66 registers
    constexpr int NBD = MX_BORDER_FLOATS + 2;
    __shared__ float s_border[K == 8 ? 4 * NBD : 4];
    const TimeArgs<float> &a = m.t;
    const int lane = threadIdx.x & 63;
    float *my_border = s_border + (K == 8 ? (threadIdx.x >> 6) * NBD : 0);
    int cur_b = -1;
    h16x8 ahi = {}, alo = {};
    float inv = 0.f, gh = 0.f, cx = 0.f, cy = 0.f;
    bool wide = false;
    MxPad pad;
    for (;;) {
        unsigned long long tk = 0;
        if (lane == 0) tk = atomicAdd(a.queue, 1ull);
        const unsigned long long t0 = __shfl(tk, 0);
        const uint32_t tlo = __builtin_amdgcn_readfirstlane((uint32_t)t0);
        const uint32_t thi = __builtin_amdgcn_readfirstlane((uint32_t)(t0 >> 32));
        const int64_t task = (int64_t)(((uint64_t)thi << 32) | tlo);
        if (task >= a.n_tasks) break;

        int b = 0;
        int64_t tb = 0, cb = 0, np = a.np0;
        uint64_t seed = a.seed0;
        if (a.n_u > 1) {
            int lo = 0, hi = a.n_u - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.task_off[mid] <= task) lo = mid;
                else hi = mid - 1;
            }
            b = __builtin_amdgcn_readfirstlane(lo);
            tb = a.task_off[b];
            cb = a.chunk_off[b];
            np = a.np_arr[b];
            seed = a.seed_arr[b];
        }
        if (b != cur_b) {
            const unsigned char *set = m.sets + (int64_t)b * MX_SET_BYTES;
            load_set(set, lane, ahi, alo, inv);
            gh = -m.fx.dth * inv;  // exact: inv is a power of two
            cx = -m.fx.dth * a.v0x;  // the constant drift's increment in units
            cy = -m.fx.dth * a.v0y;
            wide = !(set_vbound(set) <= m.vmax_fast);  // wave-uniform; NaN takes the wide path
            if constexpr (K == 8) {
                const float *src = reinterpret_cast<const float *>(set + MX_BORDER_OFFSET);
                wave_lds_sync();
                const float scale = reinterpret_cast<const MxHeader *>(set)->scale;
                for (int e = lane; e < NBD; e += 64) my_border[e] = src[e] * scale;
                wave_lds_sync();
            }
            cur_b = b;
        }
        const int64_t cpo = (np + 63) >> 6;
        const int64_t ch = task - tb;  // chunk within the set (< cpo * n_obs)
        const int64_t j = ch / cpo;
        const int64_t i = (ch - j * cpo) * 64 + lane;
        const uint32_t pi = (uint32_t)i + a.rp.i_off, pj = (uint32_t)j + a.rp.j_off;
        const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);

        FixCoord x, y;
        x.set(a.obs[2 * j]);
        y.set(a.obs[2 * j + 1]);

        int r = 0;
        const bool rp = MT && replay_on(a.rp);
        int64_t next = rp ? 0 : a.read_at[0];
        auto readout = [&](int64_t done) {
            if (MT && done == next) {
                if (rp) {
                    if (ch == 0 && lane == a.rp.lane) {
                        a.rp.out[2 * r] = x.value();
                        a.rp.out[2 * r + 1] = y.value();
                    }
                } else {
                    double *S = a.states + r * a.read_stride + 2 * ((cb + ch) * 64 + lane);
                    S[0] = x.value();
                    S[1] = y.value();
                }
                ++r;
                next = r < a.n_read ? (rp ? r : a.read_at[r]) : -1;
            }
        };
        readout(0);
        // the step loop, with the 32-bit or (set with a large velocity bound)
        // the 64-bit increment.  The normals come scaled by sqrt(2 kappa dt)
        // in units (m.gauss); the 32-bit step takes the constant drift's
        // increment -dt v0 in the same FMAs (cx, cy) and forms the increment
        // as -dt v + noise in one FMA on the unscaled sums, dt rounded once to
        // FP32 in units x inv_scale (relative error 2^-24 of the drift).
        auto walk = [&](auto wide_c) {
            constexpr bool WIDE = decltype(wide_c)::value;
            auto step = [&](float z0, float z1) {
                float sx, sy;
                if constexpr (K == 8) __asm__ volatile("" ::: "memory");  // re-read the borders every step
                mx_velocity_sum<K>(ahi, alo, x.at(), y.at(), sx, sy, pad, my_border);
                if constexpr (WIDE) {
                    x.advance_wide(__builtin_fmaf(sx, inv, a.v0x), z0, m.fx);
                    y.advance_wide(__builtin_fmaf(sy, inv, a.v0y), z1, m.fx);
                } else {
                    x.add(__builtin_fmaf(gh, sx, z0));
                    y.add(__builtin_fmaf(gh, sy, z1));
                }
            };
            const float ox = WIDE ? 0.f : cx, oy = WIDE ? 0.f : cy;
            int64_t n = 0;
            for (; n + 1 < a.n_steps; n += 2) {
                const U4 w = philox4x32_10_wu((uint32_t)(n >> 1), pi, pj, k0, k1);
                float z0, z1, z2, z3;
                box_muller_r2(w.x, w.y, m.gauss, ox, oy, z0, z1);
                box_muller_r2(w.z, w.w, m.gauss, ox, oy, z2, z3);
                step(z0, z1);
                readout(n + 1);
                step(z2, z3);
                readout(n + 2);
            }
            if (n < a.n_steps) {
                const U4 w = philox4x32_10_wu((uint32_t)(n >> 1), pi, pj, k0, k1);
                float z0, z1;
                box_muller_r2(w.x, w.y, m.gauss, ox, oy, z0, z1);
                step(z0, z1);
                readout(n + 1);
            }
        };
        if (wide) walk(std::true_type{});
        else walk(std::false_type{});
        if (!MT) {
            if (m.fix_states) {  // 8 bytes per particle: the fixed-point pair itself
                reinterpret_cast<uint2 *>(m.fix_states)[(cb + ch) * 64 + lane] = make_uint2(x.X, y.X);
            } else {
                double *S = a.states + 2 * ((cb + ch) * 64 + lane);
                S[0] = x.value();
                S[1] = y.value();
            }
        }
    }
}

// Teacher-forced steps and velocity at given points.  Each wave takes 64
// consecutive entries; lanes past count use the origin.
template <int K>
__global__ __launch_bounds__(256) void k_step_mx(const MxStepArgs a)
{
    __shared__ float s_border[MX_BORDER_FLOATS + 2];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool act = e < a.count;
    h16x8 ahi, alo;
    float inv;
    load_set(a.set, lane, ahi, alo, inv);
    if constexpr (K == 8) {  // border coefficients in the units of the packed ones
        if (threadIdx.x < MX_BORDER_FLOATS + 2)
            s_border[threadIdx.x] = reinterpret_cast<const float *>(a.set + MX_BORDER_OFFSET)[threadIdx.x] *
                                    reinterpret_cast<const MxHeader *>(a.set)->scale;
        __syncthreads();
    }
    FixCoord x, y;
    x.set(act ? a.X[2 * e] : 0.0);
    y.set(act ? a.X[2 * e + 1] : 0.0);
    float vx, vy;
    MxPad pad;
    mx_velocity<K>(ahi, alo, inv, x.at(), y.at(), vx, vy, pad, s_border);
    if (!act) return;
    if (a.V) {
        a.V[2 * e] = (double)(vx + a.v0x);
        a.V[2 * e + 1] = (double)(vy + a.v0y);
        return;
    }
    const uint64_t n = a.n[e];
    const U4 w = philox4x32_10((uint32_t)(n >> 1), a.i[e], a.j[e], 0u, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
    float z0, z1;
    if ((n & 1) == 0) box_muller(w.x, w.y, z0, z1);
    else box_muller(w.z, w.w, z0, z1);
    x.advance_wide(vx + a.v0x, a.fx.sq * z0, a.fx);
    y.advance_wide(vy + a.v0y, a.fx.sq * z1, a.fx);
    double nx = x.value(), ny = y.value();
    nx -= floor(nx);
    ny -= floor(ny);
    a.Y[2 * e] = nx;
    a.Y[2 * e + 1] = ny;
}

// Algorithm 2 on the disk with the matrix-core velocity (the walk, refills,
// exits and compaction of the vector kernel).
template <int K, int FK>
__global__ __launch_bounds__(256) void k_dirichlet_mx(const DirArgs<float> a, const StepConsts<float> fx,
                                                      const unsigned char *set)
{
    const int lane = threadIdx.x & 63;
    h16x8 ahi, alo;
    float inv;
    load_set(set, lane, ahi, alo, inv);
    MxPad pad;
    dirichlet_walk<float, FK, PM_DISK, DiskFix>(a, fx, [&](float xa, float ya, float &vx, float &vy) {
        mx_velocity_disk<K>(ahi, alo, inv, xa, ya, vx, vy, pad);
    });
}

// ---------------------------------------------------------------------------
// The tail of Algorithm 2 on the disk.  Walkers that the matrix-core walk
// saved to a pool (waves left with few live lanes once no fresh particle
// remains) continue one per wave, the 64 lanes sharing each step.  Lane
// 16 f + j (f = 0, 1, 2: the forms psi_F, F_x, F_y of disk_velocity; j < B)
// holds column j of form f's coefficients in FP32 and forms
// t = sum_i C_f[i][j] phi_i(x), times phi_j(y) = sin(2 pi (n_j y + ph_j)); a
// row-wise DPP sum leaves the three forms in lanes 15, 31 and 47.  Lane l
// draws the normals of Philox block b0 + l, so one draw serves 128 steps;
// each step reads its pair with a wave-uniform lane index.  Normals,
// update, exit test, source integral and cap are those of dirichlet_walk with
// DiskFix, every lane holding the walker's state and writing its exit record.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float row_shr_add(float v, int n)
{
    // v + (value of the lane n below in the same 16-lane row, 0 past its start)
    int s = 0;
    switch (n) {
    case 1: s = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x111, 0xF, 0xF, true); break;
    case 2: s = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x112, 0xF, 0xF, true); break;
    case 4: s = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x114, 0xF, 0xF, true); break;
    default: s = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x118, 0xF, 0xF, true); break;
    }
    return v + __builtin_bit_cast(float, s);
}

__device__ __forceinline__ float read_lane(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

template <int K, int FK>
__global__ __launch_bounds__(256) void k_dirichlet_tail(const DirArgs<float> a, const StepConsts<float> fx,
                                                        const double *__restrict__ coef, int row_stride)
{
    constexpr int B = 2 * K + 1;
    static_assert(K >= 1 && B <= 16, "one 16-lane row per form");
    const int lane = threadIdx.x & 63;
    const int f = lane >> 4, j = lane & 15;
    const bool act = f < 3 && j < B;
    float c[B];
#pragma unroll
    for (int i = 0; i < B; ++i) c[i] = act ? (float)coef[j * row_stride + 3 * i + f] : 0.f;
    const float nj = (float)((j + 1) >> 1), ph = (j & 1) ? 0.25f : 0.f;  // cos = sin shifted a quarter turn
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    int64_t count = (int64_t)uniform64((int64_t)*a.pin.count);
    count = count < a.pin.cap ? count : a.pin.cap;  // hand-overs past a full pool were not stored
    for (;;) {
        unsigned long long tk = 0;
        if (lane == 0) tk = atomicAdd(a.pin.head, 1ull);
        const int64_t w_ix = uniform64((int64_t)__shfl(tk, 0));
        if (w_ix >= count) break;
        const double *S = a.pin.st + w_ix * DIR_POOL_WORDS;
        DiskFix x, y;
        x.load(S[0], S[1]);
        y.load(S[2], S[3]);
        double I = S[4];
        int64_t n = (int64_t)S[5];
        const uint32_t pi = a.pin.ij[2 * w_ix], pj = a.pin.ij[2 * w_ix + 1];
        const int64_t t = (int64_t)pj * a.np + pi;
        // One Philox draw per lane gives the normals of the next 128 steps
        // (blocks b0 .. b0 + 63); the step loop's only branch is its latch.
        double xd = x.value(), yd = y.value();
        bool out = false;
        do {
            const int64_t b0 = n >> 1;
            float zr[4];
            {
                const U4 w = philox4x32_10((uint32_t)(b0 + lane), pi, pj, 0u, k0, k1);
                DiskFix::normals(w.x, w.y, fx, zr[0], zr[1]);
                DiskFix::normals(w.z, w.w, fx, zr[2], zr[3]);
            }
            int s = (int)(n - 2 * b0);
            const int64_t left = a.max_steps - n;  // steps to the cap
            const int lim = left < 128 - s ? s + (int)left : 128;
            do {
                const int src = s >> 1;
                const bool second = (s & 1) != 0;
                const float z0 = read_lane(second ? zr[2] : zr[0], src);
                const float z1 = read_lane(second ? zr[3] : zr[1], src);

                const float xs = x.at(), ys = y.at();
                float px[B];
                trig_basis<float, K>(xs, px);
                // cosine and sine entries in two sums: half the dependent chain
                float tc = c[0], ts = 0.f;
#pragma unroll
                for (int i = 1; i < B; i += 2) {
                    tc = __builtin_fmaf(c[i], px[i], tc);
                    ts = __builtin_fmaf(c[i + 1], px[i + 1], ts);
                }
                const float tj = tc + ts;
                const float pyj = j == 0 ? 1.f : __builtin_amdgcn_sinf(__builtin_fmaf(nj, ys, ph));
                float v = act ? tj * pyj : 0.f;
                v = row_shr_add(v, 1);
                v = row_shr_add(v, 2);
                v = row_shr_add(v, 4);
                v = row_shr_add(v, 8);
                const float F0 = read_lane(v, 15), FX = read_lane(v, 31), FY = read_lane(v, 47);
                const float wgt = 1.f - (xs * xs + ys * ys);
                const float chi = wgt * wgt;
                const float g4 = 4.f * wgt * F0;
                const float vx = __builtin_fmaf(chi, FX, -(g4 * ys));
                const float vy = __builtin_fmaf(chi, FY, g4 * xs);

                x.advance(vx + a.v0x, z0, fx);  // the walk's update
                y.advance(vy + a.v0y, z1, fx);
                I += source_at<FK>(a.f, xd, yd) * a.dtd;  // left point
                n += 1;
                xd = x.value();
                yd = y.value();
                // |x|^2 >= 1 tested on the unscaled integers (the 2^-30 scaling
                // is exact, so the rounding and the outcome are the same); the
                // same in every lane, so the branch is uniform
                const double Xd = (double)x.X, Yd = (double)y.X;
                out = __ballot(Xd * Xd + Yd * Yd >= 0x1p60) != 0;
                ++s;
            } while (!out & (s < lim));
        } while (!out && n < a.max_steps);
        double ex = xd, ey = yd;
        if (out) {  // radial projection onto the circle
            const double r = sqrt(xd * xd + yd * yd);
            ex = xd / r;
            ey = yd / r;
        }
        // every lane writes the same record: no lane-0 branch at the end of the
        // loop, which the compiler could merge with the next walker's lane-0
        // fetch and so split the wave around the shuffle
        write_exit_record(a.rec, t, ex, ey, I, n, out);
    }
}

// Teacher-forced steps and velocity on the disk (the walk's fixed-point
// coordinates, no wrap).
template <int K>
__global__ __launch_bounds__(256) void k_step_mx_disk(const MxStepArgs a)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool act = e < a.count;
    h16x8 ahi, alo;
    float inv;
    load_set(a.set, lane, ahi, alo, inv);
    // velocity mode evaluates at the FP32 value of any finite point; step
    // mode at the walk's fixed-point value (inside +-1.5, as for a walker)
    const double xd = act ? a.X[2 * e] : 0.0, yd = act ? a.X[2 * e + 1] : 0.0;
    DiskFix x, y;
    x.set(a.V ? 0.0 : xd);
    y.set(a.V ? 0.0 : yd);
    float vx, vy;
    MxPad pad;
    mx_velocity_disk<K>(ahi, alo, inv, a.V ? (float)xd : x.at(), a.V ? (float)yd : y.at(), vx, vy, pad);
    if (!act) return;
    if (a.V) {
        a.V[2 * e] = (double)(vx + a.v0x);
        a.V[2 * e + 1] = (double)(vy + a.v0y);
        return;
    }
    const uint64_t n = a.n[e];
    const U4 w = philox4x32_10((uint32_t)(n >> 1), a.i[e], a.j[e], 0u, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
    float z0, z1;
    if ((n & 1) == 0) DiskFix::normals(w.x, w.y, a.fx, z0, z1);
    else DiskFix::normals(w.z, w.w, a.fx, z0, z1);
    x.advance(vx + a.v0x, z0, a.fx);
    y.advance(vy + a.v0y, z1, a.fx);
    a.Y[2 * e] = x.value();
    a.Y[2 * e + 1] = y.value();
}

// Start points of the disk's fixed-point walk: a coordinate of magnitude
// 1.5 or more (or not finite) is outside what the walk represents.
__global__ __launch_bounds__(256) void k_check_disk_range(const double *__restrict__ X, int64_t count,
                                                          unsigned *flags)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const double x = X[2 * e], y = X[2 * e + 1];
    if (!(fabs(x) < 1.5 && fabs(y) < 1.5)) atomicOr(flags, PM_FLAG_RANGE);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <typename F>
static hipError_t dispatch_mx(int K, F &&f)
{
    switch (K) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 7: return f(std::integral_constant<int, 7>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_check_disk_range(const double *X, int64_t count, unsigned *flags, hipStream_t st)
{
    if (count < 1) return hipSuccess;
    hipLaunchKernelGGL(k_check_disk_range, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, X, count, flags);
    return hipGetLastError();
}

hipError_t launch_pack_mx(const MxPackArgs &a, unsigned char *out, int n_sets, hipStream_t st)
{
    if (a.K < 1 || a.K > MX_MAX_K || n_sets < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pack_mx, dim3(n_sets), dim3(256), 0, st, a, out);
    return hipGetLastError();
}

template <int K, bool MT>
static hipError_t launch_time_mx_k(const MxTimeArgs &a, int n_cu, int bpc, hipStream_t st)
{
    auto kern = k_time_mx<K, MT>;
    int per_cu = 0;
    hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0);
    if (err != hipSuccess) return err;
    if (per_cu < 1) per_cu = 1;
    if (bpc > 0 && bpc < per_cu) per_cu = bpc;
    int64_t blocks = (int64_t)per_cu * n_cu;
    const int64_t need = (a.t.n_tasks + 3) / 4;  // one task per wave
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_time_mx(const MxTimeArgs &a, int K, int n_cu, int bpc, hipStream_t st)
{
    return dispatch_mx(K, [&](auto kc) -> hipError_t {
        constexpr int KK = decltype(kc)::value;
        if (a.t.n_read > 1) return launch_time_mx_k<KK, true>(a, n_cu, bpc, st);
        return launch_time_mx_k<KK, false>(a, n_cu, bpc, st);
    });
}

hipError_t launch_step_mx(const MxStepArgs &a, int K, int domain, hipStream_t st)
{
    if (domain == PM_DISK && K > MX_MAX_K_DISK) return hipErrorInvalidValue;
    return dispatch_mx(K, [&](auto kc) -> hipError_t {
        constexpr int KK = decltype(kc)::value;
        const int64_t blocks = (a.count + 255) / 256;
        if constexpr (KK <= MX_MAX_K_DISK) {
            if (domain == PM_DISK) {
                hipLaunchKernelGGL(k_step_mx_disk<KK>, dim3((unsigned)blocks), dim3(256), 0, st, a);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL(k_step_mx<KK>, dim3((unsigned)blocks), dim3(256), 0, st, a);
        return hipGetLastError();
    });
}

hipError_t launch_dirichlet_tail(const DirArgs<float> &a, const StepConsts<float> &fx, const double *coef,
                                 int row_stride, int K, int fk, int n_cu, hipStream_t st)
{
    if (K < 1 || K > MX_MAX_K_DISK || (fk != 0 && fk != 1)) return hipErrorInvalidValue;
    return dispatch_mx(K, [&](auto kc) -> hipError_t {
        constexpr int KK = decltype(kc)::value;
        if constexpr (KK > MX_MAX_K_DISK) {
            return hipErrorInvalidValue;
        } else {
            void (*kern)(const DirArgs<float>, const StepConsts<float>, const double *, int) =
                fk == 0 ? k_dirichlet_tail<KK, 0> : k_dirichlet_tail<KK, 1>;
            int per_cu = 0;
            hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0);
            if (err != hipSuccess) return err;
            if (per_cu < 1) per_cu = 1;
            if (per_cu > 8) per_cu = 8;
            // one wave per walker at a time; waves past the pool's count exit at once
            hipLaunchKernelGGL(kern, dim3((unsigned)(per_cu * n_cu)), dim3(256), 0, st, a, fx, coef, row_stride);
            return hipGetLastError();
        }
    });
}

hipError_t launch_dirichlet_mx(const DirArgs<float> &a, const StepConsts<float> &fx, const unsigned char *set, int K,
                               int fk, int n_cu, int bpc, hipStream_t st)
{
    if (K < 1 || K > MX_MAX_K_DISK || (fk != 0 && fk != 1)) return hipErrorInvalidValue;
    return dispatch_mx(K, [&](auto kc) -> hipError_t {
        constexpr int KK = decltype(kc)::value;
        if constexpr (KK > MX_MAX_K_DISK) {
            return hipErrorInvalidValue;
        } else {
            void (*kern)(const DirArgs<float>, const StepConsts<float>, const unsigned char *) =
                fk == 0 ? k_dirichlet_mx<KK, 0> : k_dirichlet_mx<KK, 1>;
            int per_cu = 0;
            hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0);
            if (err != hipSuccess) return err;
            if (per_cu < 1) per_cu = 1;
            if (per_cu > 8) per_cu = 8;  // the compaction pools hold dirichlet_max_lanes() walkers
            if (bpc > 0 && bpc < per_cu) per_cu = bpc;
            int64_t blocks = (int64_t)per_cu * n_cu;
            const int64_t need = (a.total + 255) / 256;
            if (blocks > need) blocks = need;
            if (blocks < 1) blocks = 1;
            hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, st, a, fx, set);
            return hipGetLastError();
        }
    });
}

}  // namespace pm
