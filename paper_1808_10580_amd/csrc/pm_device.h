// pm_device.h -- device building blocks of the particle forward map (gfx950).
//
// Velocity representation.  The stream function of the paper's Fourier
// expansion (Section 4.1, eq. v_expand) over wavevectors with |k_x|,|k_y| <= K
// is a tensor product of one-dimensional trigonometric bases,
//     psi(x,y) = sum_{i,j} Psi[i][j] phi_i(x) phi_j(y),
//     phi_0 = 1, phi_{2n-1}(s) = cos(2 pi n s), phi_{2n}(s) = sin(2 pi n s),
// so each velocity component is a bilinear form phi(x)^T C phi(y) with a
// (2K+1)x(2K+1) coefficient matrix C folded once per parameter set from u.
// One bilinear form costs about B^2 fused multiply-adds (B = 2K+1) against
// 4 per wavevector for the mode-by-mode sum, i.e. roughly half the work for
// a full half-plane table, and needs only the 2 base sine/cosine pairs per
// step: the higher harmonics come from angle-addition recurrences held in
// registers.  The sines and cosines are the dominant cost the paper names
// (Section 4.1); here they are 4 hardware transcendentals per step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pm.h"

namespace pm {

struct FieldArg {
    int kind;
    int n;
    double p[PM_FIELD_MAX_PARAMS];
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The key schedule is
// uniform across a wave, so the compiler keeps it in scalar registers.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one v_mad_u64_u32 per 32x32->64 product (hi and lo words together)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        // three-input exclusive or (truth table 0x96) in one v_bitop3_b32
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// The same generator for counters (c0, c1, c2, 0) whose words c0 and c2 are
// uniform across the wave (the time kernels' step block and observation).
// Then the second round's new word 0, the first round's new word 2 and the
// product of the second and third rounds that they feed are uniform as
// well: those exclusive ors are plain ones, which the compiler places on the
// scalar unit together with the products (the three-input vector form would
// pull them onto the vector units).  Where two of the three inputs of an
// exclusive or are uniform and one is not (rounds 1-3), the uniform pair is
// combined on the scalar unit first (`su`): a vector instruction reads one
// scalar operand, so the three-input form would copy the second one into a
// vector register.  Round 0's new word 0 does not depend on c0 (the step
// block) and keeps the form the compiler hoists out of a step loop.
// Bitwise the same words as philox4x32_10.
__device__ __forceinline__ U4 philox4x32_10_wu(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t k0, uint32_t k1)
{
    uint32_t c3 = 0u;
    auto su = [](uint32_t a, uint32_t b) { return __builtin_amdgcn_readfirstlane(a ^ b); };
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        // uniform words entering round r: r = 0: all but c1; r = 1: c1, c2,
        // c3; r = 2: c0, c1, c3; r = 3: c3 (k0, k1 always)
        uint32_t n0, n2;
        if (r == 0) n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);  // no step index: hoisted
        else if (r == 1) n0 = hi1 ^ c1 ^ k0;
        else if (r == 2) n0 = hi1 ^ su(c1, k0);
        else n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
        if (r == 0) n2 = hi0 ^ c3 ^ k1;
        else if (r == 1 || r == 3) n2 = hi0 ^ su(c3, k1);
        else if (r == 2) n2 = c3 ^ su(hi0, k1);
        else n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// Box-Muller on two 24-bit uniforms: ua = ((wa>>8)+1) 2^-24 in (0,1],
// ub = (wb>>8) 2^-24 in [0,1), both exact in FP32 and FP64.
// v_log_f32 is log2, v_sin_f32/v_cos_f32 take revolutions.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float &z0, float &z1)
{
    const float ua = __builtin_fmaf((float)(wa >> 8), 0x1p-24f, 0x1p-24f);
    const float ub = (float)(wb >> 8) * 0x1p-24f;
    const float r = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(ua));
    z0 = r * __builtin_amdgcn_cosf(ub);
    z1 = r * __builtin_amdgcn_sinf(ub);
}

// The same normals times sigma plus offsets, given g = -2 ln 2 sigma^2 (FP32):
// the radius is sqrt(g log2 ua) = sigma sqrt(-2 ln ua), and each product
// with cos / sin takes its offset in the same FMA.
__device__ __forceinline__ void box_muller_r2(uint32_t wa, uint32_t wb, float g, float c0, float c1, float &z0,
                                              float &z1)
{
    const float ua = __builtin_fmaf((float)(wa >> 8), 0x1p-24f, 0x1p-24f);
    const float ub = (float)(wb >> 8) * 0x1p-24f;
    const float r = __builtin_amdgcn_sqrtf(g * __builtin_amdgcn_logf(ua));
    z0 = __builtin_fmaf(r, __builtin_amdgcn_cosf(ub), c0);
    z1 = __builtin_fmaf(r, __builtin_amdgcn_sinf(ub), c1);
}

__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double &z0, double &z1)
{
    const double ua = ((double)(wa >> 8) + 1.0) * 0x1p-24;
    const double ub = (double)(wb >> 8) * 0x1p-24;
    const double r = sqrt(-2.0 * log(ua));
    double s, c;
    sincospi(2.0 * ub, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// A 64-bit value that is the same in every lane, as a scalar (SGPR) value.
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// sin/cos of 2 pi s.
__device__ __forceinline__ void sincos_rev(float s, float &sn, float &cs)
{
    sn = __builtin_amdgcn_sinf(s);
    cs = __builtin_amdgcn_cosf(s);
}

__device__ __forceinline__ void sincos_rev(double s, double &sn, double &cs)
{
    sincospi(2.0 * s, &sn, &cs);
}

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// phi[0] = 1, phi[2n-1] = cos(2 pi n s), phi[2n] = sin(2 pi n s) for n = 1..K,
// the harmonics n >= 2 by the three-term (Chebyshev) recurrences
//   cos((n+1)t) = 2 cos t cos(nt) - cos((n-1)t),
//   sin((n+1)t) = 2 cos t sin(nt) - sin((n-1)t),
// one FMA per entry (FP32: within 2.5e-6 of the exact values up to n = 8).
template <typename T, int K>
__device__ __forceinline__ void trig_basis(T s, T *phi)
{
    phi[0] = T(1);
    if constexpr (K >= 1) {
        T s1, c1;
        sincos_rev(s, s1, c1);
        const T t = c1 + c1;
        phi[1] = c1;
        phi[2] = s1;
#pragma unroll
        for (int n = 2; n <= K; ++n) {
            phi[2 * n - 1] = fma_(t, phi[2 * n - 3], -phi[2 * n - 5 < 0 ? 0 : 2 * n - 5]);
            phi[2 * n] = n == 2 ? t * phi[2] : fma_(t, phi[2 * n - 2], -phi[2 * n - 4]);
        }
    }
}

// ---------------------------------------------------------------------------
// Particle coordinate and the Euler-Maruyama update of eq. (euler),
//   X <- X - v(X) dt + sqrt(2 kappa dt) xi.
// FP64: a double, updated as the oracle does.
// FP32: an unevaluated sum hi + lo of two floats, renormalised after every
// update (|lo| <= ulp(hi)/2), so the state carries no FP32 rounding drift;
// the velocity is evaluated at hi.  dt is split the same way so that its
// FP32 rounding does not act as a coherent bias on the drift.  On the torus
// hi is kept in [-1/2, 1/2] by subtracting rint(hi), which is exact
// (Sterbenz) because one step moves a particle by far less than 1/2.
// ---------------------------------------------------------------------------
template <typename T>
struct StepConsts {
    T dth, dtl, sq;
    T g2;  // fixed-point walks: -2 ln 2 sq^2, Box-Muller normals come out times sq
};

template <typename T>
struct Coord;

template <>
struct Coord<double> {
    double v;
    static __device__ __forceinline__ void normals(uint32_t wa, uint32_t wb, const StepConsts<double> &, double &z0,
                                                   double &z1)
    {
        box_muller(wa, wb, z0, z1);
    }
    __device__ __forceinline__ void set(double x) { v = x; }
    __device__ __forceinline__ double at() const { return v; }
    __device__ __forceinline__ double value() const { return v; }
    __device__ __forceinline__ void advance(double vel, double z, const StepConsts<double> &c)
    {
        v = __builtin_fma(-c.dth, vel, v);
        v = __builtin_fma(c.sq, z, v);
    }
    __device__ __forceinline__ void wrap() { v -= floor(v); }
    __device__ __forceinline__ void save(double &a, double &b) const
    {
        a = v;
        b = 0.0;
    }
    __device__ __forceinline__ void load(double a, double) { v = a; }
};

template <>
struct Coord<float> {
    float hi, lo;
    static __device__ __forceinline__ void normals(uint32_t wa, uint32_t wb, const StepConsts<float> &, float &z0,
                                                   float &z1)
    {
        box_muller(wa, wb, z0, z1);
    }
    __device__ __forceinline__ void set(double x)
    {
        hi = (float)x;
        lo = (float)(x - (double)hi);
    }
    __device__ __forceinline__ float at() const { return hi; }
    __device__ __forceinline__ double value() const { return (double)hi + (double)lo; }
    __device__ __forceinline__ void advance(float vel, float z, const StepConsts<float> &c)
    {
        float d = __builtin_fmaf(-c.dtl, vel, c.sq * z);
        d = __builtin_fmaf(-c.dth, vel, d);
        // two-sum hi + d = s + e exactly, then fold lo in and renormalise
        const float s = hi + d;
        const float bb = s - hi;
        float e = (hi - (s - bb)) + (d - bb);
        e += lo;
        hi = s + e;
        lo = e - (hi - s);
    }
    __device__ __forceinline__ void wrap() { hi -= __builtin_rintf(hi); }
    // exact round trip through two doubles
    __device__ __forceinline__ void save(double &a, double &b) const
    {
        a = (double)hi;
        b = (double)lo;
    }
    __device__ __forceinline__ void load(double a, double b)
    {
        hi = (float)a;
        lo = (float)b;
    }
};

// Pointer into the constant address space: uniform loads through it become
// scalar-cache loads (s_load) whose results feed VALU ops as SGPR operands.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

// Hide a pointer's value from the optimiser so that loads through it are
// issued where they stand (every step) instead of being hoisted out of the
// step loop into hundreds of registers.
template <typename P>
__device__ __forceinline__ P opaque_sgpr(P p)
{
    __asm__ volatile("" : "+s"(p));
    return p;
}

template <int K>
struct Geo {
    static constexpr int B = 2 * K + 1;            // basis size per axis
    static constexpr int RT = ((2 * B + 3) / 4) * 4;  // torus row stride (2 forms), multiple of 4
    static constexpr int RD = ((3 * B + 3) / 4) * 4;  // disk row stride (3 forms)
};

// Torus velocity: row j of C holds (Cx[i][j], Cy[i][j]) at [2i], [2i+1] with
//   v_x = d psi/dy = phi(x)^T Cx phi(y),  v_y = -d psi/dx = phi(x)^T Cy phi(y).
// By construction Cx[i][0] = 0 (no constant-in-y term survives d/dy) and
// Cy[0][j] = 0 (likewise for d/dx), which the loop skips.
// NP particles share every coefficient load.
template <typename T, int K, int NP, typename CP>
__device__ __forceinline__ void torus_velocity(CP C, const T (&phx)[NP][2 * K + 1],
                                               const T (&phy)[NP][2 * K + 1], T (&vx)[NP], T (&vy)[NP])
{
    constexpr int B = Geo<K>::B;
    constexpr int R = Geo<K>::RT;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        vx[p] = T(0);
        vy[p] = T(0);
    }
    if constexpr (K == 0) {
        return;
    } else {
        // j = 0: only the y component
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            T ty = C[2 * 1 + 1] * phx[p][1];
#pragma unroll
            for (int i = 2; i < B; ++i) ty = fma_(C[2 * i + 1], phx[p][i], ty);
            vy[p] = ty;
        }
#pragma unroll
        for (int j = 1; j < B; ++j) {
            const auto row = C + j * R;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                T tx = fma_(row[2 * 1], phx[p][1], row[0]);
                T ty = row[2 * 1 + 1] * phx[p][1];
#pragma unroll
                for (int i = 2; i < B; ++i) {
                    tx = fma_(row[2 * i], phx[p][i], tx);
                    ty = fma_(row[2 * i + 1], phx[p][i], ty);
                }
                vx[p] = fma_(tx, phy[p][j], vx[p]);
                vy[p] = fma_(ty, phy[p][j], vy[p]);
            }
        }
    }
}

// Disk velocity for psi = chi psi_F, chi = (1 - r^2)^2: row j holds
// (Psi[i][j], Cx[i][j], Cy[i][j]) at [3i..3i+2], with
//   psi_F = phi(x)^T Psi phi(y), F_x = d psi_F/dy, F_y = -d psi_F/dx.
//   v_x = d(chi psi_F)/dy = chi F_x + psi_F d chi/dy,
//   v_y = -d(chi psi_F)/dx = chi F_y - psi_F d chi/dx,
//   grad chi = -4 (1 - r^2) (x, y).
template <typename T, int K, typename CP>
__device__ __forceinline__ void disk_velocity(CP C, const T (&phx)[2 * K + 1],
                                              const T (&phy)[2 * K + 1], T x, T y, T &vx, T &vy)
{
    constexpr int B = Geo<K>::B;
    constexpr int R = Geo<K>::RD;
    T f0 = T(0), fx = T(0), fy = T(0);
#pragma unroll
    for (int j = 0; j < B; ++j) {
        const auto row = C + j * R;
        T t0 = row[0];
        T tx = row[1];
        T ty = T(0);
#pragma unroll
        for (int i = 1; i < B; ++i) {
            t0 = fma_(row[3 * i], phx[i], t0);
            tx = fma_(row[3 * i + 1], phx[i], tx);
            ty = fma_(row[3 * i + 2], phx[i], ty);
        }
        f0 = fma_(t0, phy[j], f0);
        fx = fma_(tx, phy[j], fx);
        fy = fma_(ty, phy[j], fy);
    }
    const T w = T(1) - (x * x + y * y);
    const T chi = w * w;
    const T g4 = T(4) * w * f0;  // -psi_F * dchi/d(x or y) = 4 w psi_F (x or y)
    vx = fma_(chi, fx, -(g4 * y));
    vy = fma_(chi, fy, g4 * x);
}

// ---------------------------------------------------------------------------
// Scalar fields (FP64): initial condition, boundary data and source.
// ---------------------------------------------------------------------------
__device__ inline double field_eval(const FieldArg &f, double x, double y)
{
    const double *p = f.p;
    double s = 0.0;
    switch (f.kind) {
    case PM_F_ZERO:
        return 0.0;
    case PM_F_CONST:
        return p[0];
    case PM_F_SINSIN:
        return p[0] * sinpi(2.0 * x) * sinpi(2.0 * y);
    case PM_F_FOURIER:
        for (int m = 0; m + 3 < f.n; m += 4) {
            double sn, cs;
            sincospi(2.0 * (p[m] * x + p[m + 1] * y), &sn, &cs);
            s += p[m + 2] * cs + p[m + 3] * sn;
        }
        return s;
    case PM_F_GAUSS_PERIODIC:
        for (int m = 0; m + 3 < f.n; m += 4) {
            const double cx = p[m], cy = p[m + 1], sg = p[m + 2], A = p[m + 3];
            const double inv = -1.0 / (2.0 * sg * sg);
            for (int nx = -1; nx <= 1; ++nx)
                for (int ny = -1; ny <= 1; ++ny) {
                    const double dx = x - cx - nx, dy = y - cy - ny;
                    s += A * exp((dx * dx + dy * dy) * inv);
                }
        }
        return s;
    case PM_F_COS_M_THETA:
        return cos(p[0] * atan2(y, x));
    case PM_F_EXP_LINEAR:
        return exp(p[0] * x + p[1] * y);
    case PM_F_LINEAR:
        return p[0] * x + p[1] * y + p[2];
    case PM_F_GAUSS:
        for (int m = 0; m + 3 < f.n; m += 4) {
            const double dx = x - p[m], dy = y - p[m + 1];
            s += p[m + 3] * exp(-p[m + 2] * (dx * dx + dy * dy));
        }
        return s;
    case PM_F_COS_AXES:
        return p[0] * (cos(p[1] * x) + cos(p[1] * y));
    default:
        return __builtin_nan("");
    }
}

// ---------------------------------------------------------------------------
// Wave64 reductions (FP64).  The xor butterfly is a fixed tree over the lane
// index, i.e. over the particle index within a 64-particle chunk.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace pm
