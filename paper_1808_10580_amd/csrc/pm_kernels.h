// pm_kernels.h -- kernel argument blocks and launchers shared by the kernels
// (pm_kernels.hip) and the C ABI (pm_abi.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "pm_device.h"

namespace pm {

enum : unsigned { PM_FLAG_NONFINITE = 1u, PM_FLAG_CAPPED = 2u, PM_FLAG_RANGE = 4u };
enum { PM_COEF_LDS = 0, PM_COEF_SCALAR = 1 };

struct FoldArgs {
    const int32_t *k;  // device [M][2]
    int n_modes;
    int K;
    int domain;
    int row_stride;
    const double *u;  // device [n_sets][u_stride]
    int64_t u_stride;
    int64_t coef_stride;  // elements between parameter sets in the output
};

// Path replay through the multi-readout time kernels: the launch's
// observation j and particle i run with Philox indices j + j_off and
// i + i_off, and when `lane` >= 0 every step count 0..n_read-1 is a readout
// whose position only the lane (particle offset within its chunk) `lane` of
// chunk 0 writes, to out[2 r], out[2 r + 1] (read_at[] unused).
struct Replay {
    uint32_t i_off = 0, j_off = 0;
    int lane = -1;
    double *out = nullptr;
};

__host__ __device__ __forceinline__ bool replay_on(const Replay &r) { return r.lane >= 0; }

template <typename T>
struct TimeArgs {
    const T *coef;
    int64_t coef_stride;
    const double *obs;
    int n_obs;
    int n_u;
    int64_t np0;     // n_u == 1
    uint64_t seed0;  // n_u == 1
    const int64_t *np_arr;     // n_u > 1: device [n_u]
    const uint64_t *seed_arr;  // device [n_u]
    const int64_t *task_off;   // device [n_u+1]
    const int64_t *chunk_off;  // device [n_u+1]
    int64_t n_tasks;
    int64_t n_steps;
    StepConsts<T> sc;
    T v0x, v0y;
    double *states;  // [n_read][total chunks][64][2] positions at each readout
    int64_t read_stride;  // doubles between readout slots of states
    unsigned long long *queue;
    int n_read;                      // >= 1; read_at[n_read - 1] == n_steps
    int64_t read_at[PM_MAX_READS];   // increasing step counts of the readouts
    Replay rp;                       // path replay (multi-readout kernels only)
};

struct PayArgs {
    const double *states;  // [n_read][n_chunks][64][2]
    // fixed-point final states of the small-K matrix-core kernel, [n_chunks][64]
    // (X, Y) as 32-bit fractions of the period; when set, states is unused
    const uint32_t *fix_states;
    int64_t n_chunks;      // per readout
    int n_read;
    int n_u;
    int64_t np0;
    const int64_t *np_arr;
    const int64_t *chunk_off;
    FieldArg theta0;
    double *partials;
    double *endpoints;  // nullable (n_u == 1)
    unsigned *flags;
};

// Walkers saved between the launches of a compacted Dirichlet walk.
constexpr int DIR_POOL_WORDS = 6 + PM_MAX_SOURCES;  // x hi, x lo, y hi, y lo, int f, steps, source integrals
struct DirPool {
    unsigned long long *count;  // walkers stored (a hand-over past cap is counted but not stored)
    unsigned long long *head;   // next walker to deal when the pool is the input
    double *st;                 // [cap][DIR_POOL_WORDS]
    uint32_t *ij;               // [cap][2] particle and observation index
    int64_t cap;
};

template <typename T>
struct DirArgs {
    const T *coef;
    const double *obs;
    int n_obs;
    int64_t np;
    int64_t total;
    uint64_t seed;
    int64_t max_steps;
    StepConsts<T> sc;
    T v0x, v0y;
    double dtd;
    FieldArg f;
    // [total][4], one 32-byte record per walker written once at its end: exit
    // point x, y, int_0^tau f dt, steps taken n (n for an exit, -n - 1 for a
    // capped path; exact integers)
    double *rec;
    unsigned long long *queue;
    const int *order;  // device [n_obs]: queue position -> observation (longest walks first)
    // Gaussian sources (FK = 2): per particle int_0^tau exp(-w_s |X - c_s|^2) dt
    int n_src;
    double src[PM_MAX_SOURCES][3];  // (cx, cy, w)
    double *integ_src;              // [n_src][total]
    // Compaction: mode 0 deals fresh particles, mode 1 the walkers of pin.
    // Once its input is exhausted, a wave with 1..dump_below-1 live lanes that
    // has run at least min_iters iterations in this launch saves its walkers
    // to pout and exits (dump_below = 0: run every walker to its exit).
    int mode;
    int dump_below;
    int min_iters;
    // Hand-over at a fixed step count (> 0): a walker that has taken
    // hand_steps steps is saved to pout (while it has room) and its lane takes
    // the next particle; which walkers move depends on their own steps only.
    int64_t hand_steps;
    DirPool pin, pout;
};

// One walker's exit record as a single 32-byte store (DirArgs::rec).
__device__ __forceinline__ void write_exit_record(double *rec, int64_t t, double ex, double ey, double integ,
                                                  int64_t n, bool exited)
{
    double4 r;
    r.x = ex;
    r.y = ey;
    r.z = integ;
    r.w = exited ? (double)n : -(double)n - 1.0;
    reinterpret_cast<double4 *>(rec)[t] = r;
}

struct DirPayArgs {
    int64_t total;
    double dtd;
    FieldArg g;
    const double *rec;       // the walk's exit records (DirArgs::rec)
    unsigned char *capped;   // [total] written here: 1 for a capped path
    double *pay;
    double *tau;    // [total] exit time nsteps * dt
    double *paths;  // nullable
    unsigned *flags;
};

struct FinalArgs {
    const double *partials;
    int n_obs;
    int64_t cpo;                // single parameter set
    const int64_t *chunk_off;   // batches: device [n_u+1], else nullptr
    const int64_t *np_arr;      // batches: device [n_u]
    double *mean;
    double *var;
    unsigned *flags;
};

template <typename T>
struct StepArgs {
    const T *coef;
    int domain;
    int64_t count;
    const double *X;
    const uint64_t *n;
    const uint32_t *i;
    const uint32_t *j;
    uint64_t seed;
    StepConsts<T> sc;
    T v0x, v0y;
    double *Y;
};

int row_stride(int domain, int K);

// ---------------------------------------------------------------------------
// High-wavenumber torus path (pm_hk.hip): split-FP16 matrix-core velocity.
// ---------------------------------------------------------------------------
constexpr int HK_BASIS_SHIFT = 8;  // the basis enters the products scaled by 2^8

struct HkHeader {              // start of each parameter set's coefficient block
    float inv_scale;           // 2^-(coefficient shift + HK_BASIS_SHIFT)
    float cmax;                // max |Cx|, |Cy| (FP32)
    unsigned char kt_lim[16];  // per nt stage: tiles kt >= kt_lim[nt] are zero in both components
    float pad[58];             // tiles start 256 bytes in
};
static_assert(sizeof(HkHeader) == 256, "tile alignment");

struct HkFoldArgs {
    const int32_t *index;  // device [(2K+1)^2]: mode of (k_x, k_y) at [(k_x+K)(2K+1) + k_y+K], or -1
    int n_modes;
    int K, KT, NT;
    const double *u;       // device [n_sets][u_stride]
    int64_t u_stride;
    int64_t set_bytes;     // bytes per parameter set in the output
};

struct HkTimeArgs {
    const unsigned char *frag;  // [n_u][set_bytes]
    int64_t set_bytes;
    int KT, NT, B;
    const double *obs;
    int n_obs;
    int n_u;
    int64_t np0;
    uint64_t seed0;
    const int64_t *np_arr;
    const uint64_t *seed_arr;
    const int64_t *task_off;   // one task per block: hk_particles_per_task() / 64 chunks of one set
    const int64_t *chunk_off;
    int64_t n_tasks;
    int64_t n_steps;
    StepConsts<float> sc;
    float v0x, v0y;
    double *states;            // [n_read][total chunks][64][2]
    int64_t read_stride;
    unsigned long long *queue;
    int n_read;
    int64_t read_at[PM_MAX_READS];
    Replay rp;
};

struct HkStepArgs {
    const unsigned char *frag;  // one parameter set
    int KT, NT, B;
    int64_t count;
    const double *X;
    const uint64_t *n;
    const uint32_t *i;
    const uint32_t *j;
    uint64_t seed;
    StepConsts<float> sc;
    float v0x, v0y;
    double *Y;   // step mode
    double *V;   // velocity mode when non-null (n, i, j, Y unused)
};

int hk_kt(int K);
int hk_nt(int K);
int hk_particles_per_task();  // particles one block (one task) of the time kernel serves
int64_t hk_set_bytes(int K);
hipError_t launch_fold_hk(const HkFoldArgs &a, unsigned char *out, int n_sets, hipStream_t st);
hipError_t launch_time_hk(const HkTimeArgs &a, int n_cu, hipStream_t st);
hipError_t launch_step_hk(const HkStepArgs &a, hipStream_t st);

}  // namespace pm

struct pm_ctx;
namespace pm {
// Context accessors for other parts of the library (defined in pm_abi.hip).
int ctx_device(const pm_ctx *c);
hipStream_t ctx_stream(const pm_ctx *c);
bool ctx_closed(const pm_ctx *c);
void ctx_retain(pm_ctx *c);
void ctx_drop(pm_ctx *c);

template <typename T>
hipError_t launch_fold(const FoldArgs &a, T *coef, int n_sets, hipStream_t st);
template <typename T>
hipError_t launch_time(const TimeArgs<T> &a, int K, int ppl, int src, int n_cu, int bpc, hipStream_t st);
template <typename T>
hipError_t launch_dirichlet(const DirArgs<T> &a, int K, int fk, int src, int n_cu, int bpc, int domain,
                            hipStream_t st);
hipError_t launch_dir_payoff(const DirPayArgs &a, hipStream_t st);
hipError_t launch_time_payoff(const PayArgs &a, hipStream_t st);
// A replayed path onto the torus' unit square, in place: X <- X - floor(X)
// (the same map as the endpoints of launch_time_payoff).
hipError_t launch_wrap_path(double *path, int64_t n_values, hipStream_t st);
hipError_t launch_chunk_reduce(const double *vals, int64_t np, int n_obs, double *partials,
                               unsigned *flags, hipStream_t st);
hipError_t launch_finalize(const FinalArgs &a, int n_groups, hipStream_t st);
hipError_t launch_count_capped(const unsigned char *capped, int64_t np, int n_obs, int64_t *out,
                               hipStream_t st);
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t st);
hipError_t launch_walk_order(const double *obs, int n_obs, int domain, int *order, hipStream_t st);
hipError_t launch_pool_reset(unsigned long long *in_head, unsigned long long *out_count, hipStream_t st);
int64_t dirichlet_max_lanes(int n_cu);  // resident lanes of the largest Dirichlet grid
// Central finite differences of G: parameter sets u +- h e_k and the
// Jacobian from their means.
hipError_t launch_fd_sets(const double *u, int n_coef, double h, double *U, hipStream_t st);
hipError_t launch_fd_diff(const double *U, const double *mean, int n_obs, int n_coef, double *J, hipStream_t st);
template <typename T>
hipError_t launch_step(const StepArgs<T> &a, int K, hipStream_t st);
template <typename T>
hipError_t launch_velocity(const T *coef, int domain, int K, T v0x, T v0y, int64_t count,
                           const double *X, double *V, hipStream_t st);
template <typename T>
hipError_t launch_normals(int64_t count, const uint64_t *n, const uint32_t *i, const uint32_t *j,
                          uint64_t seed, double *Z, hipStream_t st);

}  // namespace pm
