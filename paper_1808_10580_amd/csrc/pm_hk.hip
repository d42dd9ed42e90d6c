// pm_hk.hip -- the velocity field of eq. v_expand at high wavenumbers
// (|k_x|, |k_y| > 8, up to 95) on the torus, FP32 particles, on the matrix
// cores.
//
// With the axis bases phi_0 = 1, phi_{2n-1} = cos 2 pi n s, phi_{2n} =
// sin 2 pi n s (B = 2K + 1 functions) the field is two bilinear forms,
//     v_x(x, y) = phi(x)^T Cx phi(y),   v_y(x, y) = phi(x)^T Cy phi(y),
// and for a wave of 64 particles the inner products W = C^T Phi_x (B x 64
// per component) are a dense contraction of B^2 multiply-adds per particle:
// 51,842 at K = 80 against a few hundred for the basis itself.  W runs on
// v_mfma_f32_16x16x32_f16 with operands split into FP16 pairs (a = a_hi +
// a_lo), three products a_hi b_hi + a_hi b_lo + a_lo b_hi accumulated in
// FP32: a relative error of about 2^-22 per product, on par with FP32
// arithmetic.  The basis is pre-scaled by 2^8 and the coefficients by a
// power of two that puts max |C| near 2^15, so the low halves stay normal
// FP16 numbers; the result is scaled back exactly.
//
// Matrix-core layouts (16x16x32, lane l, g = l / 16):
//   A (16 rows j x 32 cols i): lane l holds C[i = 32 kt + 8 g + e][j = 16 nt + l % 16], e = 0..7
//   B (32 rows i x 16 cols p): lane l holds phi_{32 kt + 8 g + e}(x_p), particle p = 16 rb + l % 16
//   D (16 x 16, FP32):         lane l holds W[j = 16 nt + 4 g + r][p = 16 rb + l % 16], r = 0..3
// so each lane finishes the y form for one particle per row block rb and
// four j, and two butterfly steps over g complete the sums.  Particle p of a
// wave lives in lane p (the chunk layout of the time kernel).
#include "pm_kernels.h"
#include "pm_split.h"

namespace pm {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Fold: u -> split FP16 coefficient tiles.
// Psi[i][j] (coefficient of phi_i(x) phi_j(y) in psi) gathers the at most
// four modes (+-|k_x|, +-|k_y|) through a dense (2K+1)^2 index table; the
// rules are the addition theorems of the VALU fold:
//   (cos, cos) += a_m,  (sin, sin) -= sx sy a_m,  (sin, cos) += sx b_m,
//   (cos, sin) += sy b_m,   sx = sign k_x, sy = sign k_y (0 counts as +).
// ---------------------------------------------------------------------------
__device__ double hk_psi(const HkFoldArgs &a, const double *__restrict__ u, int i, int j)
{
    const int px = (i + 1) >> 1, py = (j + 1) >> 1;
    const bool si = i > 0 && !(i & 1), sj = j > 0 && !(j & 1);  // sine-type index
    const int W = 2 * a.K + 1;
    double acc = 0.0;
    for (int q = 0; q < 4; ++q) {
        const int kx = (q & 1) ? -px : px, ky = (q & 2) ? -py : py;
        if (((q & 1) && px == 0) || ((q & 2) && py == 0)) continue;  // +0 and -0 are one mode
        const int m = a.index[(kx + a.K) * W + (ky + a.K)];
        if (m < 0) continue;
        const double sx = kx < 0 ? -1.0 : 1.0, sy = ky < 0 ? -1.0 : 1.0;
        const double am = u[m], bm = u[a.n_modes + m];
        if (!si && !sj) acc += am;
        else if (si && sj) acc -= sx * sy * am;
        else if (si) acc += sx * bm;
        else acc += sy * bm;
    }
    return acc;
}

// Cx = d/dy of the Psi form, Cy = -d/dx: d/ds phi_{2n-1} = -2 pi n phi_{2n},
// d/ds phi_{2n} = 2 pi n phi_{2n-1}.
__device__ void hk_coef(const HkFoldArgs &a, const double *__restrict__ u, int i, int j, double &cx, double &cy)
{
    const double tp = 6.283185307179586476925286766559;
    cx = 0.0;
    cy = 0.0;
    if (j > 0) {
        const int n = (j + 1) >> 1;
        cx = (j & 1) ? tp * n * hk_psi(a, u, i, j + 1) : -tp * n * hk_psi(a, u, i, j - 1);
    }
    if (i > 0) {
        const int n = (i + 1) >> 1;
        cy = (i & 1) ? -tp * n * hk_psi(a, u, i + 1, j) : tp * n * hk_psi(a, u, i - 1, j);
    }
}

// One block per parameter set.  Output per set: HkHeader, then tiles
// [nt][kt][4][64][8] halves: (x hi, x lo, y hi, y lo) fragments in the A
// layout above, zero outside 0 <= i, j < B.
__global__ __launch_bounds__(256) void k_fold_hk(const HkFoldArgs a, unsigned char *__restrict__ out)
{
    __shared__ float red[256];
    __shared__ int lim[16];
    if (threadIdx.x < 16) lim[threadIdx.x] = 0;
    const int s = blockIdx.x;
    const double *__restrict__ u = a.u + (int64_t)s * a.u_stride;
    unsigned char *base = out + (int64_t)s * a.set_bytes;
    const int B = 2 * a.K + 1;
    float mx = 0.f;
    for (int e = threadIdx.x; e < B * B; e += blockDim.x) {
        double cx, cy;
        hk_coef(a, u, e / B, e % B, cx, cy);
        mx = fmaxf(mx, fmaxf(fabsf((float)cx), fabsf((float)cy)));
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const float cmax = red[0];
    // 2^sc puts max |C| in [2^14, 2^15)
    int sc = 0;
    if (cmax > 0.f) {
        int ex;
        frexpf(cmax, &ex);  // cmax = f 2^ex, f in [0.5, 1)
        sc = 15 - ex;
    }
    HkHeader *h = reinterpret_cast<HkHeader *>(base);
    if (threadIdx.x == 0) {
        h->inv_scale = ldexpf(1.f, -(sc + HK_BASIS_SHIFT));
        h->cmax = cmax;
    }
    _Float16 *t = reinterpret_cast<_Float16 *>(base + sizeof(HkHeader));
    const int KT = a.KT, NT = a.NT;
    const int64_t n_half = (int64_t)NT * KT * 4 * 64 * 8;
    for (int64_t q = threadIdx.x; q < n_half / 2; q += blockDim.x) {
        // q enumerates (nt, kt, comp, lane, e) with the hi / lo pair together
        const int e = (int)(q & 7);
        const int lane = (int)((q >> 3) & 63);
        const int64_t r = q >> 9;
        const int comp = (int)(r & 1);
        const int64_t tile = r >> 1;  // nt * KT + kt
        const int kt = (int)(tile % KT), nt = (int)(tile / KT);
        const int i = 32 * kt + 8 * (lane >> 4) + e;
        const int j = 16 * nt + (lane & 15);
        float v = 0.f;
        if (i < B && j < B) {
            double cx, cy;
            hk_coef(a, u, i, j, cx, cy);
            v = ldexpf((float)(comp ? cy : cx), sc);
        }
        const _Float16 hi = (_Float16)v;
        const _Float16 lo = (_Float16)(v - (float)hi);
        const int64_t frag = ((tile * 4) + 2 * comp) * 64 + lane;  // hi fragment; lo is the next one
        t[frag * 8 + e] = hi;
        t[(frag + 64) * 8 + e] = lo;
        if (v != 0.f) atomicMax(&lim[nt], kt + 1);
    }
    __syncthreads();
    if (threadIdx.x < 16) h->kt_lim[threadIdx.x] = (unsigned char)lim[threadIdx.x];
}

// ---------------------------------------------------------------------------
// Basis values at a double-float coordinate s = sh + sl.
// The phase n s mod 1 is formed without losing the low bits: p = n sh is
// rounded, its error e = fma(n, sh, -p) is exact, p - rint(p) is exact, and
// the small terms e + n sl are added last.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float hk_phase(int n, float sh, float sl)
{
    const float fn = (float)n;
    const float p = fn * sh;
    const float e = __builtin_fmaf(fn, sh, -p);
    const float f = p - __builtin_rintf(p);
    return f + __builtin_fmaf(fn, sl, e);
}

// A lane needs, per particle, runs of D consecutive frequencies n0 + d that
// repeat every S frequencies (one run per tile).  The first run and the
// rotation by S come from the hardware sine/cosine; each further run follows
// from the two before it by the three-term recurrences
//   cos((n+S)t) = 2 cos(St) cos(nt) - cos((n-S)t),
//   sin((n+S)t) = 2 cos(St) sin(nt) - sin((n-S)t),
// one FMA per value, the run before the first one being the first rotated
// back by S (angle subtraction).  A run may start scaled by a power of two
// (the x basis), which every later run then carries exactly.
template <int D>
struct Run {
    float c[D], s[D];    // frequencies n0 + d + mS
    float pc[D], ps[D];  // frequencies n0 + d + (m - 1)S
    float t;             // 2 cos(St)
};

template <int D>
__device__ __forceinline__ void run_init(Run<D> &r, int n0, int S, float sh, float sl, float scale)
{
    float sS, cS;
    sincos_rev(hk_phase(S, sh, sl), sS, cS);
    r.t = cS + cS;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        float sn, cn;
        sincos_rev(hk_phase(n0 + d, sh, sl), sn, cn);
        r.c[d] = cn * scale;
        r.s[d] = sn * scale;
        r.pc[d] = __builtin_fmaf(r.c[d], cS, r.s[d] * sS);
        r.ps[d] = __builtin_fmaf(r.s[d], cS, -(r.c[d] * sS));
    }
}

template <int D>
__device__ __forceinline__ void run_next(Run<D> &r)
{
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const float c = __builtin_fmaf(r.t, r.c[d], -r.pc[d]);
        const float s = __builtin_fmaf(r.t, r.s[d], -r.ps[d]);
        r.pc[d] = r.c[d];
        r.ps[d] = r.s[d];
        r.c[d] = c;
        r.s[d] = s;
    }
}

// ---------------------------------------------------------------------------
// Velocity of the particle held by each thread of the block (all 256 threads
// take part; threads without a particle pass any finite position).  The
// coefficient tiles of one nt stage (KT x 4 fragments of 1 KB) are staged in
// LDS, double-buffered: while the matrix cores work on stage nt, the block's
// loads of stage nt+1 are in flight.
// ---------------------------------------------------------------------------
template <int KT, int RB>
__device__ __forceinline__ void hk_velocity_block(const unsigned char *__restrict__ set, int NT, int B, float xh,
                                                  float xl, float yh, float yl, f16x8 *__restrict__ lds, float &vx,
                                                  float &vy)
{
    constexpr int FR = KT * 4 * 64;  // fragments (f16x8) per nt stage
    constexpr int PER = FR / 256;    // per thread: KT
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int g = lane >> 4, c = lane & 15;
    const HkHeader *h = reinterpret_cast<const HkHeader *>(set);
    const float inv = h->inv_scale;
    const f16x8 *__restrict__ tiles = reinterpret_cast<const f16x8 *>(set + sizeof(HkHeader));

    // Stage nt of the tiles goes straight from global memory into LDS buffer
    // buf (global_load_lds: each lane writes 16 bytes at a wave-uniform base
    // plus 16 x lane).  Fragment tid + 256 q of a stage belongs to tile
    // kt = q; tiles at or past kt_lim[nt] are zero and are neither loaded nor
    // used.
    auto stage_load = [&](int nt_, int buf) {
        const int lim = h->kt_lim[nt_];
        const int wv = tid >> 6;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (q < lim) {
                const f16x8 *src = tiles + (int64_t)nt_ * FR + 256 * q + tid;
                f16x8 *dst = lds + buf * FR + 256 * q + 64 * wv;
                __builtin_amdgcn_global_load_lds((const void *)src, (__attribute__((address_space(3))) void *)dst, 16,
                                                 0, 0);
            }
        }
    };
    stage_load(0, 0);

    // positions of the particles this lane serves in the contraction
    float pxh[RB], pxl[RB], pyh[RB], pyl[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int src = 16 * rb + c;
        pxh[rb] = __shfl(xh, src);
        pxl[rb] = __shfl(xl, src);
        pyh[rb] = __shfl(yh, src);
        pyl[rb] = __shfl(yl, src);
    }
    // B operands: phi_{32 kt + 8 g + e}(x) x 2^8 split into FP16 pairs;
    // frequencies 16 kt + 4 g + d (d = 0..4).  The run starts scaled by 2^8
    // and the recurrence coefficient 2 cos(16t) is unscaled, so every value
    // carries the scale exactly (a power of two commutes with each rounding).
    f16x8 bh[KT][RB], bl[KT][RB];
    constexpr float SCL = (float)(1 << HK_BASIS_SHIFT);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        Run<5> rx;
        run_init(rx, 4 * g, 16, pxh[rb], pxl[rb], SCL);
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            if (kt) run_next(rx);
            const int i0 = 32 * kt + 8 * g;
            float o[8];
            o[0] = (i0 == 0) ? SCL : rx.s[0];
            o[1] = rx.c[1];
            o[2] = rx.s[1];
            o[3] = rx.c[2];
            o[4] = rx.s[2];
            o[5] = rx.c[3];
            o[6] = rx.s[3];
            o[7] = rx.c[4];
            // entries past B meet zero coefficient rows, so their (finite)
            // values do not matter and need no masking
            uint32_t hw[4], lw[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) split_pair(o[2 * d], o[2 * d + 1], hw[d], lw[d]);
            bh[kt][rb] = __builtin_bit_cast(f16x8, (u32x4){hw[0], hw[1], hw[2], hw[3]});
            bl[kt][rb] = __builtin_bit_cast(f16x8, (u32x4){lw[0], lw[1], lw[2], lw[3]});
        }
    }
    // y basis runs: frequencies 8 nt + 2 g + d (d = 0..2), one run per rb
    Run<3> ry[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) run_init(ry[rb], 2 * g, 8, pyh[rb], pyl[rb], 1.f);

    __builtin_amdgcn_s_waitcnt(0);  // vmcnt(0) expcnt(0) lgkmcnt(0): stage 0 is in LDS
    __syncthreads();

    float ax[RB], ay[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) ax[rb] = ay[rb] = 0.f;
    for (int nt = 0; nt < NT; ++nt) {
        const f16x8 *__restrict__ cur = lds + (nt & 1) * FR;
        const int lcur = h->kt_lim[nt];
        // buffer (nt+1)&1 was last read in iteration nt-1, before its barrier
        if (nt + 1 < NT) stage_load(nt + 1, (nt + 1) & 1);
        f32x4 dx[RB], dy[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            dx[rb] = (f32x4){0.f, 0.f, 0.f, 0.f};
            dy[rb] = (f32x4){0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            if (kt >= lcur) break;  // zero tiles (uniform)
            const f16x8 *f = cur + kt * 4 * 64 + lane;
            const f16x8 xhi = f[0], xlo = f[64], yhi = f[128], ylo = f[192];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                dx[rb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(xhi, bh[kt][rb], dx[rb], 0, 0, 0);
                dx[rb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(xhi, bl[kt][rb], dx[rb], 0, 0, 0);
                dx[rb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(xlo, bh[kt][rb], dx[rb], 0, 0, 0);
                dy[rb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(yhi, bh[kt][rb], dy[rb], 0, 0, 0);
                dy[rb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(yhi, bl[kt][rb], dy[rb], 0, 0, 0);
                dy[rb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ylo, bh[kt][rb], dy[rb], 0, 0, 0);
            }
        }
        // y form: rows j = 16 nt + 4 g + r of particle 16 rb + c
        const int j0 = 16 * nt + 4 * g;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            if (nt) run_next(ry[rb]);
            float f4[4];
            f4[0] = (j0 == 0) ? 1.f : ry[rb].s[0];
            f4[1] = ry[rb].c[1];
            f4[2] = ry[rb].s[1];
            f4[3] = ry[rb].c[2];
            // rows j >= B of D are exact zeros (zero coefficient columns)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ax[rb] = __builtin_fmaf(dx[rb][r], f4[r], ax[rb]);
                ay[rb] = __builtin_fmaf(dy[rb][r], f4[r], ay[rb]);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);  // stage nt+1 has landed in LDS
        __syncthreads();
    }
    // sum over the four row groups (fixed butterfly: identical in every lane)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        ax[rb] += __shfl_xor(ax[rb], 16);
        ay[rb] += __shfl_xor(ay[rb], 16);
        ax[rb] += __shfl_xor(ax[rb], 32);
        ay[rb] += __shfl_xor(ay[rb], 32);
    }
    // lane l = 16 g + c holds particle 16 (g mod RB) + c (with RB = 2 the
    // upper half of the wave mirrors the lower half)
    const int rsel = g % RB;
    float sx = ax[0], sy = ay[0];
#pragma unroll
    for (int rb = 1; rb < RB; ++rb)
        if (rsel == rb) {
            sx = ax[rb];
            sy = ay[rb];
        }
    vx = sx * inv;
    vy = sy * inv;
}

// ---------------------------------------------------------------------------
// Algorithm 1 with the matrix-core velocity, persistent.  A task is up to 4
// consecutive 64-particle chunks of one parameter set, one per wave of the
// block (the chunk layout and the reduction of the VALU time kernel); a wave
// without a chunk walks a dummy particle so that the block stays in step.
// States are read out at the step counts read_at[].
// ---------------------------------------------------------------------------
template <int KT, int RB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RB == 2 ? 2 : 1))) void k_time_hk(
    const HkTimeArgs a)
{
    __shared__ f16x8 lds[2 * KT * 4 * 64];
    __shared__ unsigned long long s_task;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    for (;;) {
        if (threadIdx.x == 0) s_task = atomicAdd(a.queue, 1ull);
        __syncthreads();
        const unsigned long long tk = s_task;
        __syncthreads();
        const uint32_t tlo = __builtin_amdgcn_readfirstlane((uint32_t)tk);
        const uint32_t thi = __builtin_amdgcn_readfirstlane((uint32_t)(tk >> 32));
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
        // a wave serves 16 RB particles: RB = 4 one chunk, RB = 2 half a chunk
        // (lanes 32..63 then mirror lanes 0..31)
        constexpr int WPC = 4 / RB;  // waves per chunk
        const int64_t cpo = (np + 63) >> 6;
        const int64_t nch = cpo * a.n_obs;
        const int64_t ch = (task - tb) * (4 / WPC) + w / WPC;  // this wave's chunk within the set
        const int part = (w % WPC) * 16 * RB + (lane % (16 * RB));  // particle offset within the chunk
        const bool wave_on = ch < nch;
        const bool writer = wave_on && lane < 16 * RB;
        const int64_t chv = wave_on ? ch : 0;
        const int64_t j = chv / cpo;
        const int64_t i = (chv - j * cpo) * 64 + part;
        const uint32_t pi = (uint32_t)i + a.rp.i_off, pj = (uint32_t)j + a.rp.j_off;
        const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
        const unsigned char *set = a.frag + (int64_t)b * a.set_bytes;

        Coord<float> x, y;
        x.set(a.obs[2 * j]);
        y.set(a.obs[2 * j + 1]);

        auto step = [&](float z0, float z1) {
            float vx, vy;
            hk_velocity_block<KT, RB>(set, a.NT, a.B, x.hi, x.lo, y.hi, y.lo, lds, vx, vy);
            x.advance(vx + a.v0x, z0, a.sc);
            y.advance(vy + a.v0y, z1, a.sc);
            x.wrap();
            y.wrap();
        };
        int r = 0;
        const bool rp = replay_on(a.rp);
        int64_t next = rp ? 0 : a.read_at[0];
        auto readout = [&](int64_t done) {
            if (done == next) {
                if (rp) {
                    if (writer && ch == 0 && part == a.rp.lane) {
                        a.rp.out[2 * r] = x.value();
                        a.rp.out[2 * r + 1] = y.value();
                    }
                } else if (writer) {
                    double *S = a.states + r * a.read_stride + 2 * ((cb + ch) * 64 + part);
                    S[0] = x.value();
                    S[1] = y.value();
                }
                ++r;
                next = r < a.n_read ? (rp ? r : a.read_at[r]) : -1;
            }
        };
        readout(0);
        int64_t n = 0;
        for (; n + 1 < a.n_steps; n += 2) {
            const U4 wd = philox4x32_10((uint32_t)(n >> 1), pi, pj, 0u, k0, k1);
            float z0, z1, z2, z3;
            box_muller(wd.x, wd.y, z0, z1);
            box_muller(wd.z, wd.w, z2, z3);
            step(z0, z1);
            readout(n + 1);
            step(z2, z3);
            readout(n + 2);
        }
        if (n < a.n_steps) {
            const U4 wd = philox4x32_10((uint32_t)(n >> 1), pi, pj, 0u, k0, k1);
            float z0, z1;
            box_muller(wd.x, wd.y, z0, z1);
            step(z0, z1);
            readout(n + 1);
        }
    }
}

// Teacher-forced steps and velocity at given points, through
// hk_velocity_block.  Each block takes 256 consecutive entries; threads past
// count use the origin.
template <int KT>
__global__ __launch_bounds__(256) void k_step_hk(const HkStepArgs a)
{
    __shared__ f16x8 lds[2 * KT * 4 * 64];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = e < a.count;
    Coord<float> x, y;
    x.set(act ? a.X[2 * e] : 0.0);
    y.set(act ? a.X[2 * e + 1] : 0.0);
    float vx, vy;
    hk_velocity_block<KT, 4>(a.frag, a.NT, a.B, x.hi, x.lo, y.hi, y.lo, lds, vx, vy);
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
    x.advance(vx + a.v0x, z0, a.sc);
    y.advance(vy + a.v0y, z1, a.sc);
    double nx = x.value(), ny = y.value();
    nx -= floor(nx);
    ny -= floor(ny);
    a.Y[2 * e] = nx;
    a.Y[2 * e + 1] = ny;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
int hk_kt(int K) { return (2 * K + 1 + 31) / 32; }
int hk_nt(int K) { return (2 * K + 1 + 15) / 16; }

int64_t hk_set_bytes(int K)
{
    return (int64_t)sizeof(HkHeader) + (int64_t)hk_nt(K) * hk_kt(K) * 4 * 64 * 8 * (int64_t)sizeof(_Float16);
}

// Row blocks (16 particles) per wave in the time kernel: 2 keeps two waves per
// SIMD resident, so one wave's vector work overlaps the other's matrix work.
#ifndef HK_RB
#define HK_RB 2
#endif

int hk_particles_per_task() { return 4 * 16 * HK_RB; }

hipError_t launch_fold_hk(const HkFoldArgs &a, unsigned char *out, int n_sets, hipStream_t st)
{
    hipLaunchKernelGGL(k_fold_hk, dim3(n_sets), dim3(256), 0, st, a, out);
    return hipGetLastError();
}

template <typename F>
static hipError_t dispatch_kt(int KT, F &&f)
{
    switch (KT) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_time_hk(const HkTimeArgs &a, int n_cu, hipStream_t st)
{
    return dispatch_kt(a.KT, [&](auto kc) -> hipError_t {
        constexpr int KT = decltype(kc)::value;
        auto kern = k_time_hk<KT, HK_RB>;
        int per_cu = 0;
        hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0);
        if (err != hipSuccess) return err;
        if (per_cu < 1) per_cu = 1;
        int64_t blocks = (int64_t)per_cu * n_cu;
        if (blocks > a.n_tasks) blocks = a.n_tasks;  // one task per block
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, st, a);
        return hipGetLastError();
    });
}

hipError_t launch_step_hk(const HkStepArgs &a, hipStream_t st)
{
    return dispatch_kt(a.KT, [&](auto kc) -> hipError_t {
        constexpr int KT = decltype(kc)::value;
        const int64_t blocks = (a.count + 255) / 256;
        hipLaunchKernelGGL(k_step_hk<KT>, dim3((unsigned)blocks), dim3(256), 0, st, a);
        return hipGetLastError();
    });
}

}  // namespace pm
