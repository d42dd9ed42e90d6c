// pm_mx.h -- argument blocks and launchers of the small-K matrix-core
// velocity engine (pm_mx.hip), shared with the C ABI (pm_abi.hip).
#pragma once

#include "pm_kernels.h"

namespace pm {

// ---------------------------------------------------------------------------
// Small-K torus path (pm_mx.hip): split-FP16 matrix-core velocity for
// 1 <= K <= MX_MAX_K.  Basis entries 0..15 of each axis go through the
// 16-entry tile; at K = 8 (B = 17) the entry-16 row and column of the
// coefficient matrices are added on the vector units.
// ---------------------------------------------------------------------------
constexpr int MX_MAX_K = 8;
constexpr int MX_MAX_K_DISK = 4;         // the disk's three forms: 3 x 9 rows of the 32-row tile
// Power-of-two scale of the x basis in the products (0: unscaled; the matrix
// cores take FP16 subnormal low halves exactly).
constexpr int MX_BASIS_SHIFT = 0;
// Per parameter set: 64-byte header, A hi, A lo (64 lanes x 16 B each), then
// MX_BORDER_FLOATS border coefficients (K = 8): C_c[16][j] for c = x, y and
// j = 0..16, then C_c[i][16] x 2^-MX_BASIS_SHIFT for i = 0..15.
constexpr int MX_BORDER_FLOATS = 2 * 17 + 2 * 16;
constexpr int64_t MX_BORDER_OFFSET = 2112;
constexpr int64_t MX_SET_BYTES = MX_BORDER_OFFSET + 4 * (MX_BORDER_FLOATS + 2);
static_assert(MX_SET_BYTES % 16 == 0, "set alignment");

// Tile layout of the small-K torus and disk paths.  Basis entry 0 is the
// constant S (x basis) or 1 (y basis); entries 2v + 1, 2v + 2 (v = 0..K-1)
// are cos and sin of harmonic v + 1.
//
// x basis, the 16-entry contraction dimension: slot s = 8 h + 2 d + t sits in
// operand register d (half t) of half-wave h.  For K <= 7 register 0 of the
// lower half holds (entry 0, padding), that of the upper half padding (K <= 6)
// or the pair v = 6 (K = 7), and the pairs v = 0..5 fill registers 1..3,
// lower half first: (h, d) = (v mod 2, 1 + v / 2).  Then the constant needs
// no FP16 split and, with no varying pair beside it, no half-wave swap.  At
// K = 8 (16 entries in the tile) slot s holds entry s.  Returns -1 for
// padding.
__host__ __device__ constexpr int mx_x_entry(int K, int s)
{
    if (K >= 8) return s;
    const int h = s >> 3, d = (s & 7) >> 1, t = s & 1;
    if (d == 0) {
        if (h == 0) return t == 0 ? 0 : -1;
        return K == 7 ? 2 * 6 + 1 + t : -1;
    }
    const int v = 2 * (d - 1) + h;
    return v < K ? 2 * v + 1 + t : -1;
}

// y basis, torus: accumulator register q of half-wave h (tile row
// 8 (q / 4) + 4 h + q mod 4 of each form) meets entry 2q + 2 (h = 0) and 2q + 1
// (h = 1) for q < min(K, 7), so that one half-wave swap of the pair
// (2q + 2, 2q + 1) serves both column blocks; register min(K, 7) holds entry
// 0 (h = 0; constant 1, no swap) and padding (h = 1; entry 15 at K = 8).
// Returns -1 for padding.
__host__ __device__ constexpr int mx_y_entry(int K, int q, int h)
{
    const int m = K < 7 ? K : 7;
    if (q < m) return h == 0 ? 2 * q + 2 : 2 * q + 1;
    if (q == m) return h == 0 ? 0 : (K == 8 ? 15 : -1);
    return -1;
}

// Every basis entry the tile holds (min(2K + 1, 16) per axis) in exactly one
// slot / row, and each x register pair of one of the kinds mx_contract handles.
__host__ __device__ constexpr bool mx_layout_ok(int K)
{
    const int n = 2 * K + 1 < 16 ? 2 * K + 1 : 16;
    for (int e = 0; e < n; ++e) {
        int cx = 0, cy = 0;
        for (int s = 0; s < 16; ++s) cx += mx_x_entry(K, s) == e;
        for (int q = 0; q < 8; ++q)
            for (int h = 0; h < 2; ++h) cy += mx_y_entry(K, q, h) == e;
        if (cx != 1 || cy != 1) return false;
    }
    for (int s = 0; s < 16; ++s)
        if (mx_x_entry(K, s) >= n) return false;
    for (int d = 0; d < 4; ++d) {
        for (int h = 0; h < 2; ++h) {
            const int e0 = mx_x_entry(K, 8 * h + 2 * d), e1 = mx_x_entry(K, 8 * h + 2 * d + 1);
            if (e0 < 0 && e1 >= 0) return false;  // padding before an entry
        }
        const bool p_var = mx_x_entry(K, 2 * d) > 0 || mx_x_entry(K, 2 * d + 1) >= 0;
        const bool q_var = mx_x_entry(K, 8 + 2 * d) > 0 || mx_x_entry(K, 8 + 2 * d + 1) >= 0;
        const bool q_pad = mx_x_entry(K, 8 + 2 * d) < 0;
        if (!p_var && q_var && mx_x_entry(K, 2 * d) != 0) return false;  // padding P, varying Q
        if (p_var && !q_var && !q_pad) return false;                      // varying P, constant Q
    }
    return true;
}
static_assert(mx_layout_ok(1) && mx_layout_ok(2) && mx_layout_ok(3) && mx_layout_ok(4) && mx_layout_ok(5) &&
                  mx_layout_ok(6) && mx_layout_ok(7) && mx_layout_ok(8),
              "small-K tile layout");

struct MxHeader {
    float inv_scale;  // 2^-(coefficient shift + MX_BASIS_SHIFT)
    float cmax;       // max |Cx|, |Cy|
    float vbound;     // >= max over components of sum |C_c[i][j]| >= max |v| (torus; |phi| <= 1)
    float scale;      // 1 / inv_scale
    float pad[12];
};
static_assert(sizeof(MxHeader) == 64, "operand alignment");

struct MxPackArgs {
    const double *coef;   // FP64 coefficients of k_fold (torus or disk rows), [n_sets][coef_stride]
    int64_t coef_stride;
    int K;
    int row_stride;
    int domain;           // PM_TORUS (two forms) or PM_DISK (three)
};

// Particle coordinates of the small-K kernels are 32-bit fractions of the
// period (position = X 2^-32); their step constants come pre-scaled by 2^32.
// Usable while one step moves a particle by far less than half the period:
// the C ABI takes this engine only for sqrt(2 kappa dt) <= MX_MAX_SIGMA.
constexpr double MX_MAX_SIGMA = 0.05;
// Disk coordinates of the matrix-core walk: signed 32-bit multiples of
// 2^-MX_DISK_SHIFT (range +-2; a step is clamped to 1/2 per axis).
constexpr int MX_DISK_SHIFT = 30;

struct MxTimeArgs {
    TimeArgs<float> t;           // chunk layout, steps, readouts, outputs (t.coef, t.sc unused)
    StepConsts<float> fx;        // dt (hi + lo) and sqrt(2 kappa dt), each x 2^32
    // -2 ln 2 (2 kappa dt) 2^64: Box-Muller radius squared per log2 of the
    // uniform, so that the normals come out times sqrt(2 kappa dt) 2^32
    float gauss;
    const unsigned char *sets;   // [n_u][MX_SET_BYTES]
    // single readout: the final states as fixed-point pairs (X, Y), 8 bytes
    // per particle at [chunk][64], for the payoff kernel (t.states unused)
    uint32_t *fix_states;
    // A parameter set whose vbound is at most vmax_fast moves a particle by
    // less than 0.45 of the period per step (drift plus the largest normal),
    // so the 32-bit increment of the fixed-point update cannot overflow;
    // other sets take the 64-bit increment (exact modulo the period).
    float vmax_fast;
};

struct MxStepArgs {
    const unsigned char *set;  // one parameter set
    int64_t count;
    const double *X;
    const uint64_t *n;
    const uint32_t *i;
    const uint32_t *j;
    uint64_t seed;
    StepConsts<float> fx;  // dt (hi + lo) and sqrt(2 kappa dt), each x 2^32 (torus) or 2^MX_DISK_SHIFT (disk)
    StepConsts<float> sc;  // the same unscaled
    float v0x, v0y;
    double *Y;  // step mode
    double *V;  // velocity mode when non-null (n, i, j, Y unused)
};

// Sets PM_FLAG_RANGE in *flags unless every point of X [count][2] has
// |x|, |y| < 1.5 (the start points the disk fixed-point coordinates hold).
hipError_t launch_check_disk_range(const double *X, int64_t count, unsigned *flags, hipStream_t st);
hipError_t launch_pack_mx(const MxPackArgs &a, unsigned char *out, int n_sets, hipStream_t st);
hipError_t launch_time_mx(const MxTimeArgs &a, int K, int n_cu, int bpc, hipStream_t st);
hipError_t launch_step_mx(const MxStepArgs &a, int K, int domain, hipStream_t st);
hipError_t launch_dirichlet_mx(const DirArgs<float> &a, const StepConsts<float> &fx, const unsigned char *set, int K,
                               int fk, int n_cu, int bpc, hipStream_t st);
// The cooperative tail: walkers of a.pin (head reset to 0) run to their exit
// one per wave; coef = the FP64 disk coefficients of k_fold (row j at
// j * row_stride: Psi, Cx, Cy of entry i at 3i..3i+2).
hipError_t launch_dirichlet_tail(const DirArgs<float> &a, const StepConsts<float> &fx, const double *coef,
                                 int row_stride, int K, int fk, int n_cu, hipStream_t st);

}  // namespace pm
