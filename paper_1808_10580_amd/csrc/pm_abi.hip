// pm_abi.hip -- the extern "C" boundary of libpm.so (declared in include/pm.h).
//
// Host-side validation, workspace management and launch sequencing.  All
// arithmetic of the method runs in the kernels of pm_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "pm_mx.h"

using namespace pm;

// ---------------------------------------------------------------------------
// Fixed scratch of pm_observe_time_noalloc: one copy of this array per GPU
// (the code object's device memory), held until the process ends.  Regions,
// each 256-byte aligned: folded coefficients (the largest is the high-K
// matrix-core block of |k| <= PM_MAX_K_MFMA), matrix-core operands of the
// small-K engine, chunk partials [chunks][3] FP64, final states
// [chunks][64][2] FP64.  Host code reaches it only through the address
// hipGetSymbolAddress returns per device (noalloc_scratch).
// ---------------------------------------------------------------------------
namespace {
constexpr size_t NA_COEF_BYTES = (size_t)512 << 10;
constexpr size_t NA_MX_BYTES = (size_t)4 << 10;
constexpr size_t NA_PART_BYTES = (size_t)PM_NOALLOC_MAX_CHUNKS * 3 * sizeof(double);
constexpr size_t NA_STATE_BYTES = (size_t)PM_NOALLOC_MAX_CHUNKS * 64 * 2 * sizeof(double);
constexpr size_t NA_BYTES = NA_COEF_BYTES + NA_MX_BYTES + NA_PART_BYTES + NA_STATE_BYTES;
static_assert(NA_PART_BYTES % 256 == 0 && NA_STATE_BYTES % 256 == 0, "region alignment");
static_assert(NA_BYTES <= ((size_t)PM_NOALLOC_SCRATCH_MIB << 20), "stated scratch size");
constexpr int NA_MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[NA_MAX_DEVICES] = {};

// Device address of `scratch` on `device`, which must be the current device.
// Looked up once per device (pm_create); later calls return the kept value.
int noalloc_scratch(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= NA_MAX_DEVICES) return PM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return PM_EDEVICE;
        }
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return PM_OK;
}
}  // namespace

struct pm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 1;
    unsigned *d_flags = nullptr;
    unsigned long long *d_queue = nullptr;
    void *coef = nullptr;
    size_t coef_cap = 0;
    void *part = nullptr;
    size_t part_cap = 0;
    void *part2 = nullptr;
    size_t part2_cap = 0;
    void *pay = nullptr;
    size_t pay_cap = 0;
    void *tau = nullptr;
    size_t tau_cap = 0;
    void *capped = nullptr;
    size_t capped_cap = 0;
    void *states = nullptr;
    size_t states_cap = 0;
    void *exitp = nullptr;
    size_t exitp_cap = 0;
    void *integ = nullptr;
    size_t integ_cap = 0;
    void *nsteps = nullptr;
    size_t nsteps_cap = 0;
    void *order = nullptr;
    size_t order_cap = 0;
    void *integ_src = nullptr;  // Gaussian-source integrals [n_src][total], their partials
    size_t integ_src_cap = 0;
    void *part3 = nullptr;
    size_t part3_cap = 0;
    void *src_var = nullptr;
    size_t src_var_cap = 0;
    void *fd_u = nullptr;  // finite differences: perturbed sets, their means and variances
    size_t fd_u_cap = 0;
    void *fd_m = nullptr;
    size_t fd_m_cap = 0;
    void *meta = nullptr;
    size_t meta_cap = 0;
    int64_t *h_meta = nullptr;  // pinned staging for batch metadata
    size_t h_meta_cap = 0;
    hipEvent_t meta_ev = nullptr;
    bool meta_pending = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
    double last_steps = 0.0;
    int ppl = 0;  // explicit tuning (0 = autotuned or default)
    int src = 0;
    int bpc = 0;  // persistent blocks per CU (0 = occupancy limit)
    int dir_src = PM_COEF_SCALAR;  // Dirichlet kernel coefficient source
    int dir_bpc = 2;               // Dirichlet persistent blocks per CU (0 = occupancy)
    int dir_dump = 0;              // Dirichlet compaction (off): save waves with fewer live lanes
    int dir_launches = 8;          // ... over this many follow-up launches
    int dir_tail = 8;              // cooperative disk tail: hand over waves with fewer live lanes
    int64_t dir_hand = 0;          // ... and walkers at this step count (0: off)
    unsigned long long *tail_count = nullptr;  // walkers the last disk walk handed to the tail (device)
    void *pool = nullptr;          // compaction pools: counters, states, indices
    size_t pool_cap = 0;
    int engine = PM_ENGINE_AUTO;   // velocity engine of the FP32 torus time path
    void *mx = nullptr;            // small-K matrix-core operands [n_sets][MX_SET_BYTES]
    size_t mx_cap = 0;
    int tune_ppl[PM_MAX_K + 1] = {0};  // autotuned choice per harmonic count K
    int tune_src[PM_MAX_K + 1] = {0};
    int tune_bpc_mx[PM_MAX_K_MX + 1] = {0};  // autotuned persistent grid of the small-K matrix-core kernel
    bool capturing = false;  // recording a graph: no timing events, no host waits
    // pm_observe_time_noalloc: the per-call buffers point into the fixed
    // scratch for the duration of the call, and ensure() may not allocate
    bool no_alloc = false;
    void *scratch = nullptr;  // this device's fixed scratch (noalloc_scratch)
    // Lifetime: the caller's handle plus one reference per live problem.
    // pm_destroy releases the device resources at once; the struct itself is
    // freed with the last reference, so problems may be destroyed after it.
    int refs = 1;
    bool closed = false;
};

struct pm_graph {
    pm_ctx *owner = nullptr;
    pm_ctx *priv = nullptr;  // private workspace: never reallocated by other calls
    unsigned *priv_flags = nullptr;
    pm_problem *prob = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double steps = 0.0;
};

struct pm_problem {
    pm_ctx *ctx = nullptr;
    int refs = 1;  // the caller's handle plus one per graph that uses it
    int domain = PM_TORUS;
    int prec = PM_FP32;
    int n_modes = 0;
    int K = 0;
    int32_t *d_k = nullptr;
    double v0[2] = {0.0, 0.0};
    bool has_theta0 = false;
    FieldArg theta0{};
    bool hk = false;              // K > PM_MAX_K: matrix-core velocity (torus, FP32)
    int32_t *d_index = nullptr;   // hk: (k_x, k_y) -> mode index, [(2K+1)^2]
};

namespace {

#define PM_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return PM_EDEVICE;       \
    } while (0)

int ensure(pm_ctx *c, void **ptr, size_t *cap, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (*cap >= bytes) return PM_OK;
    if (c->no_alloc) return PM_EINVAL;  // a fixed-scratch region is too small: never allocate
    if (*ptr) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) return PM_EDEVICE;
        (void)hipFree(*ptr);
        *ptr = nullptr;
        *cap = 0;
    }
    size_t want = bytes + bytes / 4;
    if (hipMalloc(ptr, want) != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return PM_ENOMEM;
    }
    *cap = want;
    return PM_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int to_field(const pm_field *f, FieldArg *out)
{
    if (!f) return PM_EINVAL;
    if (f->kind < PM_F_ZERO || f->kind > PM_F_COS_AXES) return PM_EINVAL;
    if (f->n_params < 0 || f->n_params > PM_FIELD_MAX_PARAMS) return PM_EINVAL;
    if (f->n_params > 0 && !f->params) return PM_EINVAL;
    static const int need[] = {0, 1, 1, 4, 4, 1, 2, 3, 4, 2};
    const int n = f->n_params;
    if (n < need[f->kind]) return PM_EINVAL;
    if ((f->kind == PM_F_FOURIER || f->kind == PM_F_GAUSS_PERIODIC || f->kind == PM_F_GAUSS) && (n % 4) != 0)
        return PM_EINVAL;
    std::memset(out, 0, sizeof(*out));
    out->kind = f->kind;
    out->n = n;
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(f->params[i])) return PM_EINVAL;
        out->p[i] = f->params[i];
    }
    if (f->kind == PM_F_GAUSS_PERIODIC)
        for (int m = 0; m < n; m += 4)
            if (!(out->p[m + 2] > 0.0)) return PM_EINVAL;
    return PM_OK;
}

int64_t n_steps_of(double T, double dt) { return (int64_t)std::ceil(T / dt - 1e-9); }

// dt as hi + lo in the particle precision, and sqrt(2 kappa dt) (eq. euler with
// sigma = sqrt(2 kappa) I).
template <typename T>
StepConsts<T> step_consts(double dt, double kappa)
{
    StepConsts<T> c;
    c.dth = (T)dt;
    c.dtl = (T)(dt - (double)c.dth);
    c.sq = (T)std::sqrt(2.0 * kappa * dt);
    c.g2 = (T)0;  // unused by the floating-point coordinates
    return c;
}

// The same constants in units of 2^-32 of the period, for the fixed-point
// coordinates of the small-K matrix-core kernels.
StepConsts<float> fixed_consts(double dt, double kappa, double S = 4294967296.0)
{
    StepConsts<float> c;
    c.dth = (float)(dt * S);
    c.dtl = (float)(dt * S - (double)c.dth);
    c.sq = (float)(std::sqrt(2.0 * kappa * dt) * S);
    c.g2 = (float)(-2.0 * std::log(2.0) * (2.0 * kappa * dt) * S * S);
    return c;
}

bool mx_step_ok(double dt, double kappa) { return std::sqrt(2.0 * kappa * dt) <= MX_MAX_SIGMA; }

template <typename T>
int fold(pm_ctx *c, const pm_problem *p, const double *u, int n_sets, int64_t u_stride, T **coef_out,
         int64_t *stride_out)
{
    const int B = 2 * p->K + 1;
    const int R = row_stride(p->domain, p->K);
    const int64_t stride = (int64_t)B * R;
    int st = ensure(c, &c->coef, &c->coef_cap, (size_t)n_sets * stride * sizeof(T));
    if (st) return st;
    FoldArgs fa{};
    fa.k = p->d_k;
    fa.n_modes = p->n_modes;
    fa.K = p->K;
    fa.domain = p->domain;
    fa.row_stride = R;
    fa.u = u;
    fa.u_stride = u_stride;
    fa.coef_stride = stride;
    if (launch_fold<T>(fa, (T *)c->coef, n_sets, c->stream) != hipSuccess) return PM_EDEVICE;
    *coef_out = (T *)c->coef;
    *stride_out = stride;
    return PM_OK;
}

// Matrix-core coefficient tiles of n_sets parameter sets (high-K torus).
int fold_hk(pm_ctx *c, const pm_problem *p, const double *u, int n_sets, int64_t u_stride,
            const unsigned char **out, int64_t *set_bytes)
{
    const int64_t sb = hk_set_bytes(p->K);
    int st = ensure(c, &c->coef, &c->coef_cap, (size_t)n_sets * sb);
    if (st) return st;
    HkFoldArgs fa{};
    fa.index = p->d_index;
    fa.n_modes = p->n_modes;
    fa.K = p->K;
    fa.KT = hk_kt(p->K);
    fa.NT = hk_nt(p->K);
    fa.u = u;
    fa.u_stride = u_stride;
    fa.set_bytes = sb;
    if (launch_fold_hk(fa, (unsigned char *)c->coef, n_sets, c->stream) != hipSuccess) return PM_EDEVICE;
    *out = (const unsigned char *)c->coef;
    *set_bytes = sb;
    return PM_OK;
}

// The small-K matrix-core velocity serves FP32 torus problems with
// 1 <= K <= MX_MAX_K and FP32 disk problems with 1 <= K <= MX_MAX_K_DISK
// unless the vector engine is requested.
static_assert(PM_MAX_K_MX == MX_MAX_K && PM_MAX_K_DISK_MX == MX_MAX_K_DISK, "engine limits in pm.h");

bool use_mx(const pm_ctx *c, const pm_problem *p)
{
    if (c->engine == PM_ENGINE_VALU || p->prec != PM_FP32 || p->hk || p->K < 1) return false;
    if (p->domain == PM_TORUS) return p->K <= MX_MAX_K;
    if (p->domain == PM_DISK) return p->K <= MX_MAX_K_DISK;
    return false;
}

// FP64 fold, then the split-FP16 operands of the small-K matrix-core path.
int fold_mx(pm_ctx *c, const pm_problem *p, const double *u, int n_sets, int64_t u_stride,
            const unsigned char **out, const double **coef64 = nullptr)
{
    double *coef;
    int64_t cs;
    int st = fold<double>(c, p, u, n_sets, u_stride, &coef, &cs);
    if (st) return st;
    if (coef64) *coef64 = coef;
    st = ensure(c, &c->mx, &c->mx_cap, (size_t)n_sets * MX_SET_BYTES);
    if (st) return st;
    MxPackArgs pa{};
    pa.coef = coef;
    pa.coef_stride = cs;
    pa.K = p->K;
    pa.row_stride = row_stride(p->domain, p->K);
    pa.domain = p->domain;
    if (launch_pack_mx(pa, (unsigned char *)c->mx, n_sets, c->stream) != hipSuccess) return PM_EDEVICE;
    *out = (const unsigned char *)c->mx;
    return PM_OK;
}

// Particles per lane and coefficient source for the FP32 time kernel:
// explicit setting, else the autotuned choice for this K, else 2 / LDS.
void time_tuning(const pm_ctx *c, int K, int *ppl, int *src)
{
    if (c->ppl) {
        *ppl = c->ppl;
        *src = c->src;
    } else if (c->tune_ppl[K]) {
        *ppl = c->tune_ppl[K];
        *src = c->tune_src[K];
    } else {
        *ppl = 2;
        *src = c->src;
    }
}

// Algorithm 1 with the matrix-core velocity: one task per 64-particle chunk.
int observe_time_hk(pm_ctx *c, const pm_problem *p, int n_u, const double *u, const int64_t *nps,
                    const uint64_t *seeds, const double *obs, int n_obs, double kappa, double dte,
                    const int64_t *reads, int n_read, double *mean, double *var, double *endpoints,
                    const Replay *rp = nullptr)
{
    const int64_t Nt = reads[n_read - 1];
    const unsigned char *frag;
    int64_t sb;
    int st = fold_hk(c, p, u, n_u, 2 * (int64_t)p->n_modes, &frag, &sb);
    if (st) return st;
    HkTimeArgs a{};
    a.frag = frag;
    a.set_bytes = sb;
    a.KT = hk_kt(p->K);
    a.NT = hk_nt(p->K);
    a.B = 2 * p->K + 1;
    a.obs = obs;
    a.n_obs = n_obs;
    a.n_u = n_u;
    a.n_steps = Nt;
    a.n_read = n_read;
    for (int r = 0; r < n_read; ++r) a.read_at[r] = reads[r];
    a.sc = step_consts<float>(dte, kappa);
    a.v0x = (float)p->v0[0];
    a.v0y = (float)p->v0[1];
    a.queue = c->d_queue;
    if (rp) {  // one chunk, every step read out by one lane
        a.rp = *rp;
        a.n_read = (int)(Nt + 1);
        a.np0 = nps[0];
        a.seed0 = seeds[0];
        a.n_tasks = 1;
        if (launch_zero_u64(c->d_queue, 1, c->stream) != hipSuccess) return PM_EDEVICE;
        if (launch_time_hk(a, c->n_cu, c->stream) != hipSuccess) return PM_EDEVICE;
        return PM_OK;
    }

    PayArgs pa{};
    pa.n_u = n_u;
    pa.n_read = n_read;
    pa.theta0 = p->theta0;
    pa.endpoints = endpoints;
    pa.flags = c->d_flags;
    FinalArgs fa{};
    fa.n_obs = n_obs * n_read;
    fa.mean = mean;
    fa.var = var;
    fa.flags = c->d_flags;

    int64_t total_chunks;
    double steps = 0.0;
    if (n_u == 1) {
        const int64_t cpo = (nps[0] + 63) / 64;
        total_chunks = cpo * n_obs;
        a.np0 = nps[0];
        a.seed0 = seeds[0];
        const int64_t cpt = hk_particles_per_task() / 64;  // chunks per task (one block)
        a.n_tasks = (total_chunks + cpt - 1) / cpt;
        pa.np0 = nps[0];
        fa.cpo = cpo;
        steps = (double)nps[0] * n_obs * (double)Nt;
    } else {
        const size_t nmeta = (size_t)4 * n_u + 2;
        if (c->meta_pending && !c->capturing) {
            if (hipEventSynchronize(c->meta_ev) != hipSuccess) return PM_EDEVICE;
            c->meta_pending = false;
        }
        if (c->h_meta_cap < nmeta) {
            if (c->h_meta) (void)hipHostFree(c->h_meta);
            c->h_meta = nullptr;
            c->h_meta_cap = 0;
            if (hipHostMalloc((void **)&c->h_meta, nmeta * sizeof(int64_t)) != hipSuccess) return PM_ENOMEM;
            c->h_meta_cap = nmeta;
        }
        st = ensure(c, &c->meta, &c->meta_cap, nmeta * sizeof(int64_t));
        if (st) return st;
        int64_t *h = c->h_meta;
        int64_t *h_np = h, *h_tk = h + 2 * n_u, *h_ch = h + 3 * n_u + 1;
        uint64_t *h_sd = (uint64_t *)(h + n_u);
        h_tk[0] = 0;
        h_ch[0] = 0;
        for (int b = 0; b < n_u; ++b) {
            const int64_t nch = ((nps[b] + 63) / 64) * n_obs;
            h_np[b] = nps[b];
            h_sd[b] = seeds[b];
            h_ch[b + 1] = h_ch[b] + nch;
            const int64_t cpt = hk_particles_per_task() / 64;
            h_tk[b + 1] = h_tk[b] + (nch + cpt - 1) / cpt;
            steps += (double)nps[b] * n_obs * (double)Nt;
        }
        PM_HIP(hipMemcpyAsync(c->meta, h, nmeta * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
        if (!c->capturing) {
            PM_HIP(hipEventRecord(c->meta_ev, c->stream));
            c->meta_pending = true;
        }
        const int64_t *d = (const int64_t *)c->meta;
        a.np_arr = d;
        a.seed_arr = (const uint64_t *)(d + n_u);
        a.task_off = d + 2 * n_u;
        a.chunk_off = d + 3 * n_u + 1;
        a.n_tasks = h_tk[n_u];
        total_chunks = h_ch[n_u];
        fa.chunk_off = a.chunk_off;
        fa.np_arr = a.np_arr;
        pa.chunk_off = a.chunk_off;
        pa.np_arr = a.np_arr;
    }
    st = ensure(c, &c->part, &c->part_cap, (size_t)n_read * total_chunks * 3 * sizeof(double));
    if (st) return st;
    st = ensure(c, &c->states, &c->states_cap, (size_t)n_read * total_chunks * 64 * 2 * sizeof(double));
    if (st) return st;
    a.states = (double *)c->states;
    a.read_stride = total_chunks * 64 * 2;
    pa.states = a.states;
    pa.n_chunks = total_chunks;
    pa.partials = (double *)c->part;
    fa.partials = pa.partials;

    if (launch_zero_u64(c->d_queue, 1, c->stream) != hipSuccess) return PM_EDEVICE;
    if (!c->capturing) PM_HIP(hipEventRecord(c->ev0, c->stream));
    if (launch_time_hk(a, c->n_cu, c->stream) != hipSuccess) return PM_EDEVICE;
    if (!c->capturing) {
        PM_HIP(hipEventRecord(c->ev1, c->stream));
        c->timed = true;
        c->last_steps = steps;
    }
    if (launch_time_payoff(pa, c->stream) != hipSuccess) return PM_EDEVICE;
    if (launch_finalize(fa, n_u * n_obs * n_read, c->stream) != hipSuccess) return PM_EDEVICE;
    return PM_OK;
}

template <typename T>
int observe_time_core(pm_ctx *c, const pm_problem *p, int n_u, const double *u, const int64_t *nps,
                      const uint64_t *seeds, const double *obs, int n_obs, double kappa, double dte,
                      const int64_t *reads, int n_read, double *mean, double *var, double *endpoints,
                      const Replay *rp = nullptr)
{
    const int64_t Nt = reads[n_read - 1];
    if constexpr (std::is_same<T, float>::value) {
        if (p->hk)
            return observe_time_hk(c, p, n_u, u, nps, seeds, obs, n_obs, kappa, dte, reads, n_read, mean, var,
                                   endpoints, rp);
    }
    bool mx = false;
    if constexpr (std::is_same<T, float>::value) mx = use_mx(c, p) && mx_step_ok(dte, kappa);
    T *coef = nullptr;
    int64_t cstride = 0;
    const unsigned char *mx_sets = nullptr;
    int st = mx ? fold_mx(c, p, u, n_u, 2 * (int64_t)p->n_modes, &mx_sets)
                : fold<T>(c, p, u, n_u, 2 * (int64_t)p->n_modes, &coef, &cstride);
    if (st) return st;

    int ppl = 1, src = PM_COEF_LDS;  // the matrix-core kernel: one chunk per task
    if (!std::is_same<T, double>::value && !mx) {
        if (n_read > 1 || rp) {
            ppl = 2;  // the multi-readout kernel's one FP32 variant
            src = PM_COEF_SCALAR;
        } else {
            time_tuning(c, p->K, &ppl, &src);
        }
    }
    TimeArgs<T> a{};
    a.coef = coef;
    a.coef_stride = cstride;
    a.obs = obs;
    a.n_obs = n_obs;
    a.n_u = n_u;
    a.n_steps = Nt;
    a.n_read = n_read;
    for (int r = 0; r < n_read; ++r) a.read_at[r] = reads[r];
    a.sc = step_consts<T>(dte, kappa);
    a.v0x = (T)p->v0[0];
    a.v0y = (T)p->v0[1];
    a.queue = c->d_queue;
    if (rp) {  // one chunk, every step read out by one lane
        a.rp = *rp;
        a.n_read = (int)(Nt + 1);
        a.np0 = nps[0];
        a.seed0 = seeds[0];
        a.n_tasks = 1;
    }

    PayArgs pa{};
    pa.n_u = n_u;
    pa.n_read = n_read;
    pa.theta0 = p->theta0;
    pa.endpoints = endpoints;
    pa.flags = c->d_flags;

    FinalArgs fa{};
    fa.n_obs = n_obs * n_read;  // n_u == 1 when n_read > 1: rows (r, j)
    fa.mean = mean;
    fa.var = var;
    fa.flags = c->d_flags;

    int64_t total_chunks;
    double steps = 0.0;
    if (rp) {
        total_chunks = 0;
    } else if (n_u == 1) {
        const int64_t cpo = (nps[0] + 63) / 64;
        total_chunks = cpo * n_obs;
        a.np0 = nps[0];
        a.seed0 = seeds[0];
        a.n_tasks = (total_chunks + ppl - 1) / ppl;
        pa.np0 = nps[0];
        fa.cpo = cpo;
        steps = (double)nps[0] * n_obs * (double)Nt;
    } else {
        // metadata: np[n_u] seed[n_u] task_off[n_u+1] chunk_off[n_u+1]
        const size_t nmeta = (size_t)4 * n_u + 2;
        if (c->meta_pending && !c->capturing) {
            if (hipEventSynchronize(c->meta_ev) != hipSuccess) return PM_EDEVICE;
            c->meta_pending = false;
        }
        if (c->h_meta_cap < nmeta) {
            if (c->h_meta) (void)hipHostFree(c->h_meta);
            c->h_meta = nullptr;
            c->h_meta_cap = 0;
            if (hipHostMalloc((void **)&c->h_meta, nmeta * sizeof(int64_t)) != hipSuccess) return PM_ENOMEM;
            c->h_meta_cap = nmeta;
        }
        st = ensure(c, &c->meta, &c->meta_cap, nmeta * sizeof(int64_t));
        if (st) return st;
        int64_t *h = c->h_meta;
        int64_t *h_np = h, *h_tk = h + 2 * n_u, *h_ch = h + 3 * n_u + 1;
        uint64_t *h_sd = (uint64_t *)(h + n_u);
        h_tk[0] = 0;
        h_ch[0] = 0;
        for (int b = 0; b < n_u; ++b) {
            const int64_t cpo = (nps[b] + 63) / 64;
            const int64_t nch = cpo * n_obs;
            h_np[b] = nps[b];
            h_sd[b] = seeds[b];
            h_ch[b + 1] = h_ch[b] + nch;
            h_tk[b + 1] = h_tk[b] + (nch + ppl - 1) / ppl;
            steps += (double)nps[b] * n_obs * (double)Nt;
        }
        PM_HIP(hipMemcpyAsync(c->meta, h, nmeta * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
        if (!c->capturing) {
            PM_HIP(hipEventRecord(c->meta_ev, c->stream));
            c->meta_pending = true;
        }
        const int64_t *d = (const int64_t *)c->meta;
        a.np_arr = d;
        a.seed_arr = (const uint64_t *)(d + n_u);
        a.task_off = d + 2 * n_u;
        a.chunk_off = d + 3 * n_u + 1;
        a.n_tasks = h_tk[n_u];
        total_chunks = h_ch[n_u];
        fa.chunk_off = a.chunk_off;
        fa.np_arr = a.np_arr;
        pa.chunk_off = a.chunk_off;
        pa.np_arr = a.np_arr;
    }
    if (!rp) {
        st = ensure(c, &c->part, &c->part_cap, (size_t)n_read * total_chunks * 3 * sizeof(double));
        if (st) return st;
        st = ensure(c, &c->states, &c->states_cap, (size_t)n_read * total_chunks * 64 * 2 * sizeof(double));
        if (st) return st;
        a.states = (double *)c->states;
        a.read_stride = total_chunks * 64 * 2;
    }
    pa.states = a.states;
    pa.n_chunks = total_chunks;
    pa.partials = (double *)c->part;
    fa.partials = pa.partials;

    if (launch_zero_u64(c->d_queue, 1, c->stream) != hipSuccess) return PM_EDEVICE;
    if (!c->capturing && !rp) PM_HIP(hipEventRecord(c->ev0, c->stream));
    hipError_t le;
    if constexpr (std::is_same<T, float>::value) {
        if (mx) {
            MxTimeArgs ma{};
            ma.t = a;
            ma.fx = fixed_consts(dte, kappa);
            ma.gauss = ma.fx.g2;
            ma.sets = mx_sets;
            if (n_read == 1 && !rp) {  // single readout: 8-byte fixed-point final states
                ma.fix_states = (uint32_t *)c->states;
                pa.fix_states = ma.fix_states;
            }
            ma.vmax_fast = (float)((0.45 - 5.9 * std::sqrt(2.0 * kappa * dte)) / dte -
                                   std::max(std::fabs(p->v0[0]), std::fabs(p->v0[1])));
            le = launch_time_mx(ma, p->K, c->n_cu, c->bpc ? c->bpc : c->tune_bpc_mx[p->K], c->stream);
        } else {
            le = launch_time<T>(a, p->K, ppl, src, c->n_cu, c->bpc, c->stream);
        }
    } else {
        le = launch_time<T>(a, p->K, ppl, src, c->n_cu, c->bpc, c->stream);
    }
    if (le != hipSuccess) return PM_EDEVICE;
    if (rp) return PM_OK;
    if (!c->capturing) {
        PM_HIP(hipEventRecord(c->ev1, c->stream));
        c->timed = true;
        c->last_steps = steps;
    }
    if (launch_time_payoff(pa, c->stream) != hipSuccess) return PM_EDEVICE;
    if (launch_finalize(fa, n_u * n_obs * n_read, c->stream) != hipSuccess) return PM_EDEVICE;
    return PM_OK;
}

// Single observation time T: N_t = ceil(T/dt) uniform steps of T/N_t.
template <typename T>
int observe_time_impl(pm_ctx *c, const pm_problem *p, int n_u, const double *u, const int64_t *nps,
                      const uint64_t *seeds, const double *obs, int n_obs, double kappa, double T_,
                      double dt, double *mean, double *var, double *endpoints)
{
    const int64_t Nt = n_steps_of(T_, dt);
    return observe_time_core<T>(c, p, n_u, u, nps, seeds, obs, n_obs, kappa, T_ / (double)Nt, &Nt, 1, mean,
                                var, endpoints);
}

template <typename T>
int observe_dirichlet_impl(pm_ctx *c, const pm_problem *p, const double *u, const FieldArg &f,
                           const FieldArg &g, const double *obs, int n_obs, double kappa, double dt,
                           int64_t np, uint64_t seed, int64_t max_steps, double *mean, double *var,
                           double *tau_mean, double *tau_var, int64_t *n_capped, double *paths,
                           int n_src = 0, const double *src = nullptr, double *src_mean = nullptr)
{
    // the disk's FP32 walk runs the matrix-core velocity where it applies
    bool mx = false;
    if constexpr (std::is_same<T, float>::value)
        mx = p->domain == PM_DISK && n_src == 0 && use_mx(c, p) && mx_step_ok(dt, kappa);
    T *coef = nullptr;
    int64_t cstride = 0;
    const unsigned char *mx_set = nullptr;
    const double *coef64 = nullptr;
    int st = mx ? fold_mx(c, p, u, 1, 2 * (int64_t)p->n_modes, &mx_set, &coef64)
                : fold<T>(c, p, u, 1, 2 * (int64_t)p->n_modes, &coef, &cstride);
    if (st) return st;
    const int64_t total = np * n_obs;
    if ((st = ensure(c, &c->pay, &c->pay_cap, total * sizeof(double)))) return st;
    if ((st = ensure(c, &c->tau, &c->tau_cap, total * sizeof(double)))) return st;
    if ((st = ensure(c, &c->exitp, &c->exitp_cap, 4 * total * sizeof(double)))) return st;  // exit records
    if ((st = ensure(c, &c->capped, &c->capped_cap, total))) return st;
    const int64_t cpo = (np + 63) / 64;
    if ((st = ensure(c, &c->part, &c->part_cap, cpo * n_obs * 3 * sizeof(double)))) return st;
    if ((st = ensure(c, &c->part2, &c->part2_cap, cpo * n_obs * 3 * sizeof(double)))) return st;

    // zero, constant and linear sources run as f = p0 x + p1 y + p2 in the walk;
    // Gaussian sources (n_src > 0) integrate one integral per source
    int fk = 1;
    FieldArg fpoly{};
    if (n_src > 0) {
        fk = 2;
        if ((st = ensure(c, &c->integ_src, &c->integ_src_cap, (size_t)n_src * total * sizeof(double)))) return st;
        if ((st = ensure(c, &c->part3, &c->part3_cap, cpo * n_obs * 3 * sizeof(double)))) return st;
        if ((st = ensure(c, &c->src_var, &c->src_var_cap, (size_t)n_obs * sizeof(double)))) return st;
    } else if (f.kind == PM_F_ZERO || f.kind == PM_F_CONST || f.kind == PM_F_LINEAR) {
        fk = 0;
        fpoly.kind = PM_F_LINEAR;
        fpoly.n = 3;
        if (f.kind == PM_F_CONST) fpoly.p[2] = f.p[0];
        if (f.kind == PM_F_LINEAR) {
            fpoly.p[0] = f.p[0];
            fpoly.p[1] = f.p[1];
            fpoly.p[2] = f.p[2];
        }
    }

    // Deal the walks with the longest expected exit time first (points nearest
    // the centre first; computed on the device, no synchronisation)
    if ((st = ensure(c, &c->order, &c->order_cap, (size_t)n_obs * sizeof(int)))) return st;
    if (launch_walk_order(obs, n_obs, p->domain, (int *)c->order, c->stream) != hipSuccess) return PM_EDEVICE;

    DirArgs<T> a{};
    a.coef = coef;
    a.obs = obs;
    a.order = (const int *)c->order;
    a.n_obs = n_obs;
    a.np = np;
    a.total = total;
    a.seed = seed;
    a.max_steps = max_steps;
    a.sc = step_consts<T>(dt, kappa);
    a.dtd = dt;
    a.v0x = (T)p->v0[0];
    a.v0y = (T)p->v0[1];
    a.f = fk == 0 ? fpoly : f;
    a.rec = (double *)c->exitp;
    a.queue = c->d_queue;
    a.n_src = n_src;
    for (int q = 0; q < n_src; ++q)
        for (int e = 0; e < 3; ++e) a.src[q][e] = src[3 * q + e];
    a.integ_src = (double *)c->integ_src;

    // Compaction pools (two, used alternately): walkers saved by one launch
    // are dealt densely by the next; the last launch runs every walker out.
    // The cooperative tail (matrix-core disk walk, sources without Gaussians)
    // takes the place of the follow-up launches: one launch runs the saved
    // walkers one per wave.
    const bool tail = mx && fk <= 1 && (c->dir_tail > 0 || c->dir_hand > 0);
    const int n_follow = tail ? 0 : (c->dir_dump > 0 ? c->dir_launches : 0);
    DirPool pools[2] = {};
    c->tail_count = nullptr;
    if (n_follow > 0 || tail) {
        const int64_t cap = std::min<int64_t>(total, dirichlet_max_lanes(c->n_cu));
        const size_t st_bytes = (size_t)cap * DIR_POOL_WORDS * sizeof(double);
        const size_t ij_bytes = (size_t)cap * 2 * sizeof(uint32_t);
        const size_t bytes = 4 * sizeof(unsigned long long) + 2 * (st_bytes + ij_bytes);
        if ((st = ensure(c, &c->pool, &c->pool_cap, bytes))) return st;
        char *base = (char *)c->pool;
        for (int q = 0; q < 2; ++q) {
            pools[q].count = (unsigned long long *)base + 2 * q;
            pools[q].head = (unsigned long long *)base + 2 * q + 1;
            pools[q].st = (double *)(base + 4 * sizeof(unsigned long long) + q * st_bytes);
            pools[q].ij = (uint32_t *)(base + 4 * sizeof(unsigned long long) + 2 * st_bytes + q * ij_bytes);
            pools[q].cap = cap;
        }
        if (launch_zero_u64((unsigned long long *)base, 4, c->stream) != hipSuccess) return PM_EDEVICE;
    }
    a.min_iters = 1024;
    a.hand_steps = tail ? c->dir_hand : 0;

    if (launch_zero_u64(c->d_queue, 1, c->stream) != hipSuccess) return PM_EDEVICE;
    if (mx && launch_check_disk_range(obs, n_obs, c->d_flags, c->stream) != hipSuccess) return PM_EDEVICE;
    PM_HIP(hipEventRecord(c->ev0, c->stream));
    a.mode = 0;
    a.dump_below = tail ? c->dir_tail : (n_follow > 0 ? c->dir_dump : 0);
    a.pout = pools[0];
    auto launch = [&]() -> hipError_t {
        if constexpr (std::is_same<T, float>::value) {
            if (mx)
                return launch_dirichlet_mx(a, fixed_consts(dt, kappa, std::ldexp(1.0, MX_DISK_SHIFT)), mx_set, p->K, fk,
                                           c->n_cu, c->dir_bpc, c->stream);
        }
        return launch_dirichlet<T>(a, p->K, fk, c->dir_src, c->n_cu, c->dir_bpc, p->domain, c->stream);
    };
    if (launch() != hipSuccess) return PM_EDEVICE;
    if constexpr (std::is_same<T, float>::value) {
        if (tail) {
            a.mode = 1;
            a.pin = pools[0];
            a.dump_below = 0;
            a.hand_steps = 0;
            if (launch_pool_reset(pools[0].head, pools[1].count, c->stream) != hipSuccess) return PM_EDEVICE;
            if (launch_dirichlet_tail(a, fixed_consts(dt, kappa, std::ldexp(1.0, MX_DISK_SHIFT)), coef64,
                                      row_stride(p->domain, p->K), p->K, fk, c->n_cu, c->stream) != hipSuccess)
                return PM_EDEVICE;
            c->tail_count = pools[0].count;
        }
    }
    for (int r = 1; r <= n_follow; ++r) {
        a.mode = 1;
        a.pin = pools[(r - 1) & 1];
        a.pout = pools[r & 1];
        a.dump_below = r < n_follow ? c->dir_dump : 0;
        if (launch_pool_reset(a.pin.head, a.pout.count, c->stream) != hipSuccess) return PM_EDEVICE;
        if (launch() != hipSuccess) return PM_EDEVICE;
    }
    PM_HIP(hipEventRecord(c->ev1, c->stream));
    c->timed = true;
    c->last_steps = -1.0;  // counted by the caller from the exit steps

    DirPayArgs pa{};
    pa.total = total;
    pa.dtd = dt;
    pa.g = g;
    pa.rec = a.rec;
    pa.tau = (double *)c->tau;
    pa.capped = (unsigned char *)c->capped;
    pa.pay = (double *)c->pay;
    pa.paths = paths;
    pa.flags = c->d_flags;
    if (launch_dir_payoff(pa, c->stream) != hipSuccess) return PM_EDEVICE;
    if (launch_chunk_reduce(pa.pay, np, n_obs, (double *)c->part, c->d_flags, c->stream)) return PM_EDEVICE;
    if (launch_chunk_reduce(pa.tau, np, n_obs, (double *)c->part2, c->d_flags, c->stream)) return PM_EDEVICE;
    FinalArgs fa{};
    fa.n_obs = n_obs;
    fa.cpo = cpo;
    fa.flags = c->d_flags;
    fa.partials = (const double *)c->part;
    fa.mean = mean;
    fa.var = var;
    if (launch_finalize(fa, n_obs, c->stream) != hipSuccess) return PM_EDEVICE;
    fa.partials = (const double *)c->part2;
    fa.mean = tau_mean;
    fa.var = tau_var;
    if (launch_finalize(fa, n_obs, c->stream) != hipSuccess) return PM_EDEVICE;
    if (launch_count_capped(pa.capped, np, n_obs, n_capped, c->stream) != hipSuccess) return PM_EDEVICE;
    for (int q = 0; q < n_src; ++q) {  // mean of each source integral per observation
        const double *vals = (const double *)c->integ_src + (size_t)q * total;
        if (launch_chunk_reduce(vals, np, n_obs, (double *)c->part3, c->d_flags, c->stream)) return PM_EDEVICE;
        fa.partials = (const double *)c->part3;
        fa.mean = src_mean + (size_t)q * n_obs;
        fa.var = (double *)c->src_var;
        if (launch_finalize(fa, n_obs, c->stream) != hipSuccess) return PM_EDEVICE;
    }
    return PM_OK;
}

bool bad_ptr(const void *p) { return p == nullptr; }

void ctx_release(pm_ctx *c)
{
    if (--c->refs == 0) delete c;
}

bool ctx_ok(const pm_ctx *c, const pm_problem *p) { return c && p && p->ctx == c && !c->closed; }

}  // namespace

namespace pm {
int ctx_device(const pm_ctx *c) { return c->device; }
hipStream_t ctx_stream(const pm_ctx *c) { return c->stream; }
bool ctx_closed(const pm_ctx *c) { return c->closed; }
void ctx_retain(pm_ctx *c) { c->refs++; }
void ctx_drop(pm_ctx *c) { ctx_release(c); }
}  // namespace pm

extern "C" {

const char *pm_strerror(int s)
{
    switch (s) {
    case PM_OK: return "ok";
    case PM_EINVAL: return "invalid argument";
    case PM_ENOMEM: return "device allocation failed";
    case PM_EDEVICE: return "HIP runtime error";
    case PM_ENONFINITE: return "non-finite payoff or statistic";
    case PM_ECAPPED: return "a Dirichlet path reached max_steps";
    case PM_EUNSUPPORTED: return "outside the compiled kernel set";
    default: return "unknown status";
    }
}

int pm_create(pm_ctx **out, int device, void *stream)
{
    if (!out) return PM_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return PM_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return PM_EDEVICE;
    pm_ctx *c = new (std::nothrow) pm_ctx();
    if (!c) return PM_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)stream;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return PM_EDEVICE;
    }
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    const int sst = noalloc_scratch(device, &c->scratch);
    if (sst != PM_OK && sst != PM_EUNSUPPORTED) {
        delete c;
        return sst;
    }
    if (hipMalloc((void **)&c->d_flags, 64) != hipSuccess ||
        hipMalloc((void **)&c->d_queue, 64) != hipSuccess ||
        hipMemset(c->d_flags, 0, 64) != hipSuccess ||
        hipMemset(c->d_queue, 0, 64) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipEventCreateWithFlags(&c->meta_ev, hipEventDisableTiming) != hipSuccess) {
        pm_destroy(c);
        return PM_EDEVICE;
    }
    *out = c;
    return PM_OK;
}

void pm_destroy(pm_ctx *c)
{
    if (!c || c->closed) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    void *bufs[] = {c->d_flags, c->d_queue, c->coef, c->part, c->part2, c->pay, c->tau, c->capped,
                    c->meta, c->states, c->exitp, c->integ, c->nsteps, c->order, c->fd_u, c->fd_m,
                    c->integ_src, c->part3, c->src_var, c->pool, c->mx};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (c->h_meta) (void)hipHostFree(c->h_meta);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->meta_ev) (void)hipEventDestroy(c->meta_ev);
    c->closed = true;
    ctx_release(c);
}

int pm_set_stream(pm_ctx *c, void *stream)
{
    if (!c || c->closed) return PM_EINVAL;
    c->stream = (hipStream_t)stream;
    return PM_OK;
}

int pm_set_tuning(pm_ctx *c, int ppl, int src)
{
    if (!c || c->closed) return PM_EINVAL;
    if (!(ppl == 0 || (ppl >= 1 && ppl <= 4))) return PM_EINVAL;
    if (!(src == 0 || src == 1)) return PM_EINVAL;
    c->ppl = ppl;
    c->src = src;
    return PM_OK;
}

int pm_set_velocity_engine(pm_ctx *c, int engine)
{
    if (!c || c->closed) return PM_EINVAL;
    if (engine != PM_ENGINE_AUTO && engine != PM_ENGINE_VALU && engine != PM_ENGINE_MFMA) return PM_EINVAL;
    c->engine = engine;
    return PM_OK;
}

int pm_problem_create(pm_ctx *c, pm_problem **out, int domain, int n_modes, const int32_t *k,
                      const double *v0, const pm_field *theta0, int prec)
{
    if (!c || !out) return PM_EINVAL;
    *out = nullptr;
    if (c->closed) return PM_EINVAL;
    if (domain != PM_TORUS && domain != PM_DISK && domain != PM_SQUARE) return PM_EINVAL;
    if (prec != PM_FP32 && prec != PM_FP64) return PM_EINVAL;
    if (n_modes < 0 || (n_modes > 0 && !k)) return PM_EINVAL;
    int K = 0;
    for (int m = 0; m < n_modes; ++m) {
        const int ax = k[2 * m] < 0 ? -k[2 * m] : k[2 * m];
        const int ay = k[2 * m + 1] < 0 ? -k[2 * m + 1] : k[2 * m + 1];
        if (ax > PM_MAX_K_MFMA || ay > PM_MAX_K_MFMA) return PM_EUNSUPPORTED;
        if (ax > K) K = ax;
        if (ay > K) K = ay;
    }
    const bool hk = K > PM_MAX_K;
    if (hk && (domain != PM_TORUS || prec != PM_FP32)) return PM_EUNSUPPORTED;
    std::vector<int32_t> index;
    if (hk) {
        const int W = 2 * K + 1;
        index.assign((size_t)W * W, -1);
        for (int m = 0; m < n_modes; ++m) {
            int32_t &slot = index[(size_t)(k[2 * m] + K) * W + (k[2 * m + 1] + K)];
            if (slot >= 0) return PM_EINVAL;  // a wavevector listed twice
            slot = m;
        }
    }
    if (v0 && (!std::isfinite(v0[0]) || !std::isfinite(v0[1]))) return PM_EINVAL;
    FieldArg th{};
    if (theta0) {
        if (domain != PM_TORUS) return PM_EINVAL;
        if (to_field(theta0, &th) != PM_OK) return PM_EINVAL;
    }
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    pm_problem *p = new (std::nothrow) pm_problem();
    if (!p) return PM_ENOMEM;
    p->ctx = c;
    p->domain = domain;
    p->prec = prec;
    p->n_modes = n_modes;
    p->K = K;
    if (v0) {
        p->v0[0] = v0[0];
        p->v0[1] = v0[1];
    }
    p->has_theta0 = theta0 != nullptr;
    p->theta0 = th;
    const size_t kb = (size_t)(n_modes > 0 ? n_modes : 1) * 2 * sizeof(int32_t);
    if (hipMalloc((void **)&p->d_k, kb) != hipSuccess) {
        delete p;
        return PM_ENOMEM;
    }
    if (n_modes > 0 &&
        hipMemcpy(p->d_k, k, (size_t)n_modes * 2 * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p->d_k);
        delete p;
        return PM_EDEVICE;
    }
    if (hk) {
        p->hk = true;
        const size_t ib = index.size() * sizeof(int32_t);
        if (hipMalloc((void **)&p->d_index, ib) != hipSuccess) {
            (void)hipFree(p->d_k);
            delete p;
            return PM_ENOMEM;
        }
        if (hipMemcpy(p->d_index, index.data(), ib, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(p->d_index);
            (void)hipFree(p->d_k);
            delete p;
            return PM_EDEVICE;
        }
    }
    c->refs++;
    *out = p;
    return PM_OK;
}

static void problem_release(pm_problem *p)
{
    if (--p->refs > 0) return;
    pm_ctx *c = p->ctx;
    (void)hipSetDevice(c->device);
    // the context's stream may already be gone once the context is closed
    if (!c->closed) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (p->d_k) (void)hipFree(p->d_k);
    if (p->d_index) (void)hipFree(p->d_index);
    delete p;
    ctx_release(c);
}

void pm_problem_destroy(pm_problem *p)
{
    if (!p) return;
    problem_release(p);
}

static int check_time_args(double kappa, double T, double dt)
{
    if (!(std::isfinite(kappa) && kappa >= 0.0)) return PM_EINVAL;
    if (!finite_pos(T) || !finite_pos(dt)) return PM_EINVAL;
    const int64_t Nt = n_steps_of(T, dt);
    if (Nt < 1 || Nt > ((int64_t)1 << 33)) return PM_EINVAL;
    return PM_OK;
}

int pm_observe_time(pm_ctx *c, const pm_problem *p, const double *u, const double *obs, int n_obs,
                    double kappa, double T, double dt, int64_t np, uint64_t seed, double *mean,
                    double *var, double *endpoints)
{
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (p->domain != PM_TORUS || !p->has_theta0) return PM_EINVAL;
    if ((p->n_modes > 0 && bad_ptr(u)) || bad_ptr(obs) || bad_ptr(mean) || bad_ptr(var)) return PM_EINVAL;
    if (n_obs < 1) return PM_EINVAL;
    if (np < 1 || np > ((int64_t)1 << 32)) return PM_EINVAL;
    if (check_time_args(kappa, T, dt)) return PM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    if (p->prec == PM_FP64)
        return observe_time_impl<double>(c, p, 1, u, &np, &seed, obs, n_obs, kappa, T, dt, mean, var, endpoints);
    return observe_time_impl<float>(c, p, 1, u, &np, &seed, obs, n_obs, kappa, T, dt, mean, var, endpoints);
}

int pm_observe_time_noalloc(pm_ctx *c, const pm_problem *p, const double *u, const double *obs, int n_obs,
                            double kappa, double T, double dt, int64_t np, uint64_t seed, double *mean,
                            double *var, double *endpoints)
{
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (p->domain != PM_TORUS || !p->has_theta0) return PM_EINVAL;
    if ((p->n_modes > 0 && bad_ptr(u)) || bad_ptr(obs) || bad_ptr(mean) || bad_ptr(var)) return PM_EINVAL;
    if (n_obs < 1) return PM_EINVAL;
    if (np < 1 || np > ((int64_t)1 << 32)) return PM_EINVAL;
    if (check_time_args(kappa, T, dt)) return PM_EINVAL;
    if ((np + 63) / 64 > PM_NOALLOC_MAX_CHUNKS / n_obs) return PM_EINVAL;
    if (!c->scratch) return PM_EUNSUPPORTED;  // device index beyond the scratch table
    // coefficient bytes of this problem: FP64 fold (also the small-K
    // matrix-core engine's first stage), or the high-K matrix-core block
    const int B = 2 * p->K + 1;
    const size_t coef_bytes = p->hk ? (size_t)hk_set_bytes(p->K)
                                    : (size_t)B * row_stride(p->domain, p->K) * sizeof(double);
    if (coef_bytes > NA_COEF_BYTES || (size_t)MX_SET_BYTES > NA_MX_BYTES) return PM_EUNSUPPORTED;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;

    // point the per-call buffers at the scratch for this call only
    unsigned char *base = static_cast<unsigned char *>(c->scratch);
    void *save_ptr[4] = {c->coef, c->mx, c->part, c->states};
    const size_t save_cap[4] = {c->coef_cap, c->mx_cap, c->part_cap, c->states_cap};
    c->coef = base;
    c->coef_cap = NA_COEF_BYTES;
    c->mx = base + NA_COEF_BYTES;
    c->mx_cap = NA_MX_BYTES;
    c->part = base + NA_COEF_BYTES + NA_MX_BYTES;
    c->part_cap = NA_PART_BYTES;
    c->states = base + NA_COEF_BYTES + NA_MX_BYTES + NA_PART_BYTES;
    c->states_cap = NA_STATE_BYTES;
    c->no_alloc = true;
    const int st = p->prec == PM_FP64
                       ? observe_time_impl<double>(c, p, 1, u, &np, &seed, obs, n_obs, kappa, T, dt, mean, var,
                                                   endpoints)
                       : observe_time_impl<float>(c, p, 1, u, &np, &seed, obs, n_obs, kappa, T, dt, mean, var,
                                                  endpoints);
    c->no_alloc = false;
    c->coef = save_ptr[0];
    c->mx = save_ptr[1];
    c->part = save_ptr[2];
    c->states = save_ptr[3];
    c->coef_cap = save_cap[0];
    c->mx_cap = save_cap[1];
    c->part_cap = save_cap[2];
    c->states_cap = save_cap[3];
    return st;
}

int pm_observe_time_multi(pm_ctx *c, const pm_problem *p, const double *u, const double *obs, int n_obs,
                          const int64_t *reads, int n_read, double kappa, double dt, int64_t np,
                          uint64_t seed, double *mean, double *var)
{
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (p->domain != PM_TORUS || !p->has_theta0) return PM_EINVAL;
    if ((p->n_modes > 0 && bad_ptr(u)) || bad_ptr(obs) || bad_ptr(mean) || bad_ptr(var)) return PM_EINVAL;
    if (n_obs < 1) return PM_EINVAL;
    if (np < 1 || np > ((int64_t)1 << 32)) return PM_EINVAL;
    if (!reads || n_read < 1 || n_read > PM_MAX_READS) return PM_EINVAL;
    for (int r = 0; r < n_read; ++r)
        if (reads[r] < 0 || reads[r] > ((int64_t)1 << 33) || (r > 0 && reads[r] <= reads[r - 1])) return PM_EINVAL;
    if (!(std::isfinite(kappa) && kappa >= 0.0) || !finite_pos(dt)) return PM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    if (p->prec == PM_FP64)
        return observe_time_core<double>(c, p, 1, u, &np, &seed, obs, n_obs, kappa, dt, reads, n_read, mean, var,
                                         nullptr);
    return observe_time_core<float>(c, p, 1, u, &np, &seed, obs, n_obs, kappa, dt, reads, n_read, mean, var,
                                    nullptr);
}

int pm_replay_path(pm_ctx *c, const pm_problem *p, const double *u, const double *obs, int n_obs,
                   double kappa, double T, double dt, int64_t np, uint64_t seed, int j, int64_t i, double *path)
{
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (p->domain != PM_TORUS || !p->has_theta0) return PM_EINVAL;
    if ((p->n_modes > 0 && bad_ptr(u)) || bad_ptr(obs) || bad_ptr(path)) return PM_EINVAL;
    if (n_obs < 1 || j < 0 || j >= n_obs) return PM_EINVAL;
    if (np < 1 || np > ((int64_t)1 << 32) || i < 0 || i >= np) return PM_EINVAL;
    if (check_time_args(kappa, T, dt)) return PM_EINVAL;
    const int64_t Nt = n_steps_of(T, dt);
    if (Nt >= PM_REPLAY_MAX_STEPS) return PM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    // the chunk of particle i as a one-chunk launch from x_j: Philox indices
    // (i, j) through the offsets, the same kernels and step size as the map
    Replay rp;
    rp.i_off = (uint32_t)(i - i % 64);
    rp.j_off = (uint32_t)j;
    rp.lane = (int)(i % 64);
    rp.out = path;
    const int64_t np1 = 64;
    const double dte = T / (double)Nt;
    const int st = p->prec == PM_FP64
                       ? observe_time_core<double>(c, p, 1, u, &np1, &seed, obs + 2 * (int64_t)j, 1, kappa, dte, &Nt,
                                                   1, nullptr, nullptr, nullptr, &rp)
                       : observe_time_core<float>(c, p, 1, u, &np1, &seed, obs + 2 * (int64_t)j, 1, kappa, dte, &Nt,
                                                  1, nullptr, nullptr, nullptr, &rp);
    if (st) return st;
    if (launch_wrap_path(path, 2 * (Nt + 1), c->stream) != hipSuccess) return PM_EDEVICE;
    return PM_OK;
}

int pm_jacobian_time(pm_ctx *c, const pm_problem *p, const double *u, const double *obs, int n_obs,
                     double kappa, double T, double dt, int64_t np, uint64_t seed, double h, double *J)
{
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (p->domain != PM_TORUS || !p->has_theta0) return PM_EINVAL;
    if (p->n_modes < 1 || bad_ptr(u) || bad_ptr(obs) || bad_ptr(J) || n_obs < 1) return PM_EINVAL;
    if (np < 1 || np > ((int64_t)1 << 32)) return PM_EINVAL;
    if (!finite_pos(h)) return PM_EINVAL;
    if (check_time_args(kappa, T, dt)) return PM_EINVAL;
    const int n_coef = 2 * p->n_modes;
    const int n_u = 2 * n_coef;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    int st = ensure(c, &c->fd_u, &c->fd_u_cap, (size_t)n_u * n_coef * sizeof(double));
    if (st) return st;
    if ((st = ensure(c, &c->fd_m, &c->fd_m_cap, 2 * (size_t)n_u * n_obs * sizeof(double)))) return st;
    double *U = (double *)c->fd_u, *M = (double *)c->fd_m;
    if (launch_fd_sets(u, n_coef, h, U, c->stream) != hipSuccess) return PM_EDEVICE;
    // common random numbers: every set has the same particle count and seed
    std::vector<int64_t> nps(n_u, np);
    std::vector<uint64_t> seeds(n_u, seed);
    st = p->prec == PM_FP64
             ? observe_time_impl<double>(c, p, n_u, U, nps.data(), seeds.data(), obs, n_obs, kappa, T, dt, M,
                                         M + (size_t)n_u * n_obs, nullptr)
             : observe_time_impl<float>(c, p, n_u, U, nps.data(), seeds.data(), obs, n_obs, kappa, T, dt, M,
                                        M + (size_t)n_u * n_obs, nullptr);
    if (st) return st;
    return launch_fd_diff(U, M, n_obs, n_coef, J, c->stream) == hipSuccess ? PM_OK : PM_EDEVICE;
}

int pm_observe_time_batch(pm_ctx *c, const pm_problem *p, int n_u, const double *u,
                          const int64_t *nps, const uint64_t *seeds, const double *obs, int n_obs,
                          double kappa, double T, double dt, double *mean, double *var)
{
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (p->domain != PM_TORUS || !p->has_theta0) return PM_EINVAL;
    if (n_u < 1 || !nps || !seeds) return PM_EINVAL;
    if ((p->n_modes > 0 && bad_ptr(u)) || bad_ptr(obs) || bad_ptr(mean) || bad_ptr(var)) return PM_EINVAL;
    if (n_obs < 1) return PM_EINVAL;
    for (int b = 0; b < n_u; ++b)
        if (nps[b] < 1 || nps[b] > ((int64_t)1 << 32)) return PM_EINVAL;
    if (check_time_args(kappa, T, dt)) return PM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    if (p->prec == PM_FP64)
        return observe_time_impl<double>(c, p, n_u, u, nps, seeds, obs, n_obs, kappa, T, dt, mean, var, nullptr);
    return observe_time_impl<float>(c, p, n_u, u, nps, seeds, obs, n_obs, kappa, T, dt, mean, var, nullptr);
}

int pm_observe_dirichlet(pm_ctx *c, const pm_problem *p, const double *u, const pm_field *f,
                         const pm_field *g, const double *obs, int n_obs, double kappa, double dt,
                         int64_t np, uint64_t seed, int64_t max_steps, double *mean, double *var,
                         double *tau_mean, double *tau_var, int64_t *n_capped, double *paths)
{
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (p->domain != PM_DISK && p->domain != PM_SQUARE) return PM_EINVAL;
    if ((p->n_modes > 0 && bad_ptr(u)) || bad_ptr(obs) || bad_ptr(mean) || bad_ptr(var) ||
        bad_ptr(tau_mean) || bad_ptr(tau_var) || bad_ptr(n_capped))
        return PM_EINVAL;
    FieldArg ff, gg;
    if (to_field(f, &ff) != PM_OK || to_field(g, &gg) != PM_OK) return PM_EINVAL;
    if (n_obs < 1) return PM_EINVAL;
    if (np < 1 || np > ((int64_t)1 << 32)) return PM_EINVAL;
    if (!(std::isfinite(kappa) && kappa > 0.0) || !finite_pos(dt)) return PM_EINVAL;
    if (max_steps < 1 || max_steps > ((int64_t)1 << 33)) return PM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    if (p->prec == PM_FP64)
        return observe_dirichlet_impl<double>(c, p, u, ff, gg, obs, n_obs, kappa, dt, np, seed, max_steps,
                                              mean, var, tau_mean, tau_var, n_capped, paths);
    return observe_dirichlet_impl<float>(c, p, u, ff, gg, obs, n_obs, kappa, dt, np, seed, max_steps, mean,
                                         var, tau_mean, tau_var, n_capped, paths);
}

int pm_observe_dirichlet_sources(pm_ctx *c, const pm_problem *p, const double *u, const pm_field *g,
                                 const double *obs, int n_obs, double kappa, double dt, int64_t np,
                                 uint64_t seed, int64_t max_steps, int n_src, const double *sources,
                                 double *bnd_mean, double *bnd_var, double *src_mean, double *tau_mean,
                                 double *tau_var, int64_t *n_capped)
{
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (p->domain != PM_SQUARE) return PM_EUNSUPPORTED;
    if ((p->n_modes > 0 && bad_ptr(u)) || bad_ptr(obs) || bad_ptr(bnd_mean) || bad_ptr(bnd_var) ||
        bad_ptr(src_mean) || bad_ptr(tau_mean) || bad_ptr(tau_var) || bad_ptr(n_capped) || !sources)
        return PM_EINVAL;
    if (n_src < 1 || n_src > PM_MAX_SOURCES) return PM_EINVAL;
    for (int q = 0; q < 3 * n_src; ++q)
        if (!std::isfinite(sources[q])) return PM_EINVAL;
    FieldArg gg, zero{};
    zero.kind = PM_F_ZERO;
    if (to_field(g, &gg) != PM_OK) return PM_EINVAL;
    if (n_obs < 1) return PM_EINVAL;
    if (np < 1 || np > ((int64_t)1 << 32)) return PM_EINVAL;
    if (!(std::isfinite(kappa) && kappa > 0.0) || !finite_pos(dt)) return PM_EINVAL;
    if (max_steps < 1 || max_steps > ((int64_t)1 << 33)) return PM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    if (p->prec == PM_FP64)
        return observe_dirichlet_impl<double>(c, p, u, zero, gg, obs, n_obs, kappa, dt, np, seed, max_steps,
                                              bnd_mean, bnd_var, tau_mean, tau_var, n_capped, nullptr, n_src,
                                              sources, src_mean);
    return observe_dirichlet_impl<float>(c, p, u, zero, gg, obs, n_obs, kappa, dt, np, seed, max_steps, bnd_mean,
                                         bnd_var, tau_mean, tau_var, n_capped, nullptr, n_src, sources, src_mean);
}

// Teacher-forced steps (Y) or velocities (V) through the matrix-core field.
static int step_hk(pm_ctx *c, const pm_problem *p, const double *u, int64_t count, const double *X,
                   const uint64_t *n, const uint32_t *i, const uint32_t *j, double kappa, double dt,
                   uint64_t seed, double *Y, double *V)
{
    const unsigned char *frag;
    int64_t sb;
    int st = fold_hk(c, p, u, 1, 2 * (int64_t)p->n_modes, &frag, &sb);
    if (st) return st;
    HkStepArgs a{};
    a.frag = frag;
    a.KT = hk_kt(p->K);
    a.NT = hk_nt(p->K);
    a.B = 2 * p->K + 1;
    a.count = count;
    a.X = X;
    a.n = n;
    a.i = i;
    a.j = j;
    a.seed = seed;
    a.sc = step_consts<float>(dt, kappa);
    a.v0x = (float)p->v0[0];
    a.v0y = (float)p->v0[1];
    a.Y = Y;
    a.V = V;
    return launch_step_hk(a, c->stream) == hipSuccess ? PM_OK : PM_EDEVICE;
}

static int step_mx(pm_ctx *c, const pm_problem *p, const double *u, int64_t count, const double *X,
                   const uint64_t *n, const uint32_t *i, const uint32_t *j, double kappa, double dt,
                   uint64_t seed, double *Y, double *V)
{
    const unsigned char *set;
    int st = fold_mx(c, p, u, 1, 2 * (int64_t)p->n_modes, &set);
    if (st) return st;
    MxStepArgs a{};
    a.set = set;
    a.count = count;
    a.X = X;
    a.n = n;
    a.i = i;
    a.j = j;
    a.seed = seed;
    a.fx = fixed_consts(dt, kappa, p->domain == PM_DISK ? std::ldexp(1.0, MX_DISK_SHIFT) : 4294967296.0);
    a.sc = step_consts<float>(dt, kappa);
    a.v0x = (float)p->v0[0];
    a.v0y = (float)p->v0[1];
    a.Y = Y;
    a.V = V;
    if (p->domain == PM_DISK && Y && launch_check_disk_range(X, count, c->d_flags, c->stream) != hipSuccess)
        return PM_EDEVICE;
    return launch_step_mx(a, p->K, p->domain, c->stream) == hipSuccess ? PM_OK : PM_EDEVICE;
}

int pm_step(pm_ctx *c, const pm_problem *p, const double *u, int64_t count, const double *X,
            const uint64_t *n, const uint32_t *i, const uint32_t *j, double kappa, double dt,
            uint64_t seed, double *Y)
{
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (count < 0) return PM_EINVAL;
    if (count == 0) return PM_OK;
    if ((p->n_modes > 0 && bad_ptr(u)) || bad_ptr(X) || bad_ptr(n) || bad_ptr(i) || bad_ptr(j) || bad_ptr(Y))
        return PM_EINVAL;
    if (!(std::isfinite(kappa) && kappa >= 0.0) || !finite_pos(dt)) return PM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    if (p->hk) return step_hk(c, p, u, count, X, n, i, j, kappa, dt, seed, Y, nullptr);
    if (use_mx(c, p) && mx_step_ok(dt, kappa))
        return step_mx(c, p, u, count, X, n, i, j, kappa, dt, seed, Y, nullptr);
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        T *coef;
        int64_t cs;
        int st = fold<T>(c, p, u, 1, 2 * (int64_t)p->n_modes, &coef, &cs);
        if (st) return st;
        StepArgs<T> a{};
        a.coef = coef;
        a.domain = p->domain;
        a.count = count;
        a.X = X;
        a.n = n;
        a.i = i;
        a.j = j;
        a.seed = seed;
        a.sc = step_consts<T>(dt, kappa);
        a.v0x = (T)p->v0[0];
        a.v0y = (T)p->v0[1];
        a.Y = Y;
        return launch_step<T>(a, p->K, c->stream) == hipSuccess ? PM_OK : PM_EDEVICE;
    };
    return p->prec == PM_FP64 ? run(double{}) : run(float{});
}

int pm_velocity(pm_ctx *c, const pm_problem *p, const double *u, int64_t count, const double *X, double *V)
{
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (count < 0) return PM_EINVAL;
    if (count == 0) return PM_OK;
    if ((p->n_modes > 0 && bad_ptr(u)) || bad_ptr(X) || bad_ptr(V)) return PM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    if (p->hk) return step_hk(c, p, u, count, X, nullptr, nullptr, nullptr, 0.0, 1.0, 0, nullptr, V);
    if (use_mx(c, p)) return step_mx(c, p, u, count, X, nullptr, nullptr, nullptr, 0.0, 1.0, 0, nullptr, V);
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        T *coef;
        int64_t cs;
        int st = fold<T>(c, p, u, 1, 2 * (int64_t)p->n_modes, &coef, &cs);
        if (st) return st;
        return launch_velocity<T>(coef, p->domain, p->K, (T)p->v0[0], (T)p->v0[1], count, X, V, c->stream) ==
                       hipSuccess
                   ? PM_OK
                   : PM_EDEVICE;
    };
    return p->prec == PM_FP64 ? run(double{}) : run(float{});
}

int pm_normals(pm_ctx *c, const pm_problem *p, int64_t count, const uint64_t *n, const uint32_t *i,
               const uint32_t *j, uint64_t seed, double *Z)
{
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (count < 0) return PM_EINVAL;
    if (count == 0) return PM_OK;
    if (bad_ptr(n) || bad_ptr(i) || bad_ptr(j) || bad_ptr(Z)) return PM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    hipError_t e = p->prec == PM_FP64 ? launch_normals<double>(count, n, i, j, seed, Z, c->stream)
                                      : launch_normals<float>(count, n, i, j, seed, Z, c->stream);
    return e == hipSuccess ? PM_OK : PM_EDEVICE;
}

int pm_sync(pm_ctx *c)
{
    if (!c || c->closed) return PM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return PM_EDEVICE;
    if (hipGetLastError() != hipSuccess) return PM_EDEVICE;
    unsigned h = 0;
    if (hipMemcpy(&h, c->d_flags, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess) return PM_EDEVICE;
    if (h && hipMemset(c->d_flags, 0, sizeof(unsigned)) != hipSuccess) return PM_EDEVICE;
    if (h & PM_FLAG_RANGE) return PM_EUNSUPPORTED;
    if (h & PM_FLAG_NONFINITE) return PM_ENONFINITE;
    if (h & PM_FLAG_CAPPED) return PM_ECAPPED;
    return PM_OK;
}

int pm_last_kernel_stats(pm_ctx *c, double *ms, double *steps)
{
    if (!c || c->closed || !ms || !steps) return PM_EINVAL;
    if (!c->timed) return PM_EINVAL;
    float f = 0.f;
    if (hipEventElapsedTime(&f, c->ev0, c->ev1) != hipSuccess) return PM_EDEVICE;
    *ms = f;
    *steps = c->last_steps;
    return PM_OK;
}

int pm_set_dirichlet_source(pm_ctx *c, int src)
{
    if (!c || c->closed || !(src == PM_COEF_LDS || src == PM_COEF_SCALAR)) return PM_EINVAL;
    c->dir_src = src;
    return PM_OK;
}

int pm_set_dirichlet_blocks_per_cu(pm_ctx *c, int bpc)
{
    if (!c || c->closed || bpc < 0) return PM_EINVAL;
    c->dir_bpc = bpc;
    return PM_OK;
}

int pm_set_dirichlet_compaction(pm_ctx *c, int dump_below, int launches)
{
    if (!c || c->closed || dump_below < 0 || dump_below > 64 || launches < 0 || launches > 64) return PM_EINVAL;
    c->dir_dump = dump_below;
    c->dir_launches = launches;
    return PM_OK;
}

int pm_set_dirichlet_tail(pm_ctx *c, int live_below, int64_t hand_steps)
{
    if (!c || c->closed || live_below < 0 || live_below > 64 || hand_steps < 0 || (hand_steps & 1)) return PM_EINVAL;
    c->dir_tail = live_below;
    c->dir_hand = hand_steps;
    return PM_OK;
}

int pm_dirichlet_tail_walkers(pm_ctx *c, int64_t *walkers)
{
    if (!c || c->closed || !walkers) return PM_EINVAL;
    *walkers = 0;
    if (!c->tail_count) return PM_OK;
    unsigned long long n = 0;
    PM_HIP(hipMemcpyAsync(&n, c->tail_count, sizeof(n), hipMemcpyDeviceToHost, c->stream));
    PM_HIP(hipStreamSynchronize(c->stream));
    *walkers = (int64_t)n;
    return PM_OK;
}

int pm_set_blocks_per_cu(pm_ctx *c, int bpc)
{
    if (!c || c->closed || bpc < 0) return PM_EINVAL;
    c->bpc = bpc;
    return PM_OK;
}

int pm_graph_create_time(pm_ctx *c, const pm_problem *p, int n_u, const double *u,
                         const int64_t *nps, const uint64_t *seeds, const double *obs, int n_obs,
                         double kappa, double T, double dt, double *mean, double *var, pm_graph **out)
{
    if (!out) return PM_EINVAL;
    *out = nullptr;
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (p->domain != PM_TORUS || !p->has_theta0) return PM_EINVAL;
    if (n_u < 1 || !nps || !seeds) return PM_EINVAL;
    if ((p->n_modes > 0 && bad_ptr(u)) || bad_ptr(obs) || bad_ptr(mean) || bad_ptr(var)) return PM_EINVAL;
    if (n_obs < 1) return PM_EINVAL;
    for (int b = 0; b < n_u; ++b)
        if (nps[b] < 1 || nps[b] > ((int64_t)1 << 32)) return PM_EINVAL;
    if (check_time_args(kappa, T, dt)) return PM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;

    pm_graph *g = new (std::nothrow) pm_graph();
    if (!g) return PM_ENOMEM;
    auto fail = [&](int st) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        if (g->priv) {
            g->priv->d_flags = g->priv_flags;
            pm_destroy(g->priv);
        }
        if (g->cap) (void)hipStreamDestroy(g->cap);
        delete g;
        return st;
    };
    if (hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) != hipSuccess) return fail(PM_EDEVICE);
    int st = pm_create(&g->priv, c->device, g->cap);
    if (st) return fail(st);
    pm_ctx *q = g->priv;
    q->ppl = c->ppl;
    q->src = c->src;
    q->bpc = c->bpc;
    q->engine = c->engine;
    for (int k = 0; k <= PM_MAX_K; ++k) {
        q->tune_ppl[k] = c->tune_ppl[k];
        q->tune_src[k] = c->tune_src[k];
    }
    // graph kernels report through the owner's flags (read by pm_sync(owner))
    g->priv_flags = q->d_flags;
    q->d_flags = c->d_flags;
    auto run = [&]() -> int {
        return p->prec == PM_FP64
                   ? observe_time_impl<double>(q, p, n_u, u, nps, seeds, obs, n_obs, kappa, T, dt, mean, var, nullptr)
                   : observe_time_impl<float>(q, p, n_u, u, nps, seeds, obs, n_obs, kappa, T, dt, mean, var, nullptr);
    };
    // eager pass sizes the private workspace, so the capture allocates nothing
    if ((st = run())) return fail(st);
    if (hipStreamSynchronize(g->cap) != hipSuccess) return fail(PM_EDEVICE);
    g->steps = q->last_steps;
    q->capturing = true;
    if (hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        q->capturing = false;
        return fail(PM_EDEVICE);
    }
    st = run();
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(g->cap, &graph);
    q->capturing = false;
    g->graph = graph;
    if (st) return fail(st);
    if (ec != hipSuccess || !graph) return fail(PM_EDEVICE);
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) return fail(PM_EDEVICE);
    g->owner = c;
    c->refs++;
    g->prob = const_cast<pm_problem *>(p);
    g->prob->refs++;
    *out = g;
    return PM_OK;
}

int pm_graph_launch(pm_graph *g)
{
    if (!g || g->owner->closed) return PM_EINVAL;
    if (hipSetDevice(g->owner->device) != hipSuccess) return PM_EDEVICE;
    return hipGraphLaunch(g->exec, g->owner->stream) == hipSuccess ? PM_OK : PM_EDEVICE;
}

int pm_graph_particle_steps(const pm_graph *g, double *steps)
{
    if (!g || !steps) return PM_EINVAL;
    *steps = g->steps;
    return PM_OK;
}

void pm_graph_destroy(pm_graph *g)
{
    if (!g) return;
    pm_ctx *c = g->owner;
    (void)hipSetDevice(c->device);
    if (!c->closed) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    g->priv->d_flags = g->priv_flags;
    pm_destroy(g->priv);
    (void)hipStreamDestroy(g->cap);
    problem_release(g->prob);
    ctx_release(c);
    delete g;
}

// Fastest probe time (ms, best of two) of the forward map with the context's
// current settings.
static int probe_ms(pm_ctx *c, const pm_problem *p, const double *u, const double *obs, int n_obs, double kappa,
                    double T, double dt, int64_t np, uint64_t seed, double *tmp, double *out)
{
    double ms_best = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
        int st = observe_time_impl<float>(c, p, 1, u, &np, &seed, obs, n_obs, kappa, T, dt, tmp, tmp + n_obs,
                                          nullptr);
        if (st) return st;
        if (hipStreamSynchronize(c->stream) != hipSuccess) return PM_EDEVICE;
        float f = 0.f;
        if (hipEventElapsedTime(&f, c->ev0, c->ev1) != hipSuccess) return PM_EDEVICE;
        if (f < ms_best) ms_best = f;
    }
    *out = ms_best;
    return PM_OK;
}

int pm_autotune_time(pm_ctx *c, const pm_problem *p, const double *u, const double *obs, int n_obs,
                     double kappa, double dt, int64_t np, uint64_t seed, int n_probe_steps,
                     int *ppl_out, int *src_out, int *bpc_out, double *ms_out)
{
    if (!ctx_ok(c, p)) return PM_EINVAL;
    if (p->domain != PM_TORUS || !p->has_theta0) return PM_EINVAL;
    if ((p->n_modes > 0 && bad_ptr(u)) || bad_ptr(obs) || n_obs < 1) return PM_EINVAL;
    if (np < 1 || np > ((int64_t)1 << 32) || n_probe_steps < 1) return PM_EINVAL;
    if (!(std::isfinite(kappa) && kappa >= 0.0) || !finite_pos(dt)) return PM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return PM_EDEVICE;
    if (ppl_out) *ppl_out = 1;
    if (src_out) *src_out = PM_COEF_LDS;
    if (bpc_out) *bpc_out = 0;
    if (ms_out) *ms_out = 0.0;
    if (p->prec == PM_FP64 || p->hk) return PM_OK;  // one compiled variant
    const bool mx = use_mx(c, p) && mx_step_ok(dt, kappa);
    double *tmp = nullptr;
    if (hipMalloc((void **)&tmp, 2 * (size_t)n_obs * sizeof(double)) != hipSuccess) return PM_ENOMEM;
    const int save_ppl = c->ppl, save_src = c->src, save_bpc = c->bpc;
    const double T = n_probe_steps * dt;
    double best = 1e300;
    int st = PM_OK;
    if (mx) {
        // the matrix-core kernel: persistent blocks per compute unit (a
        // value at or above the occupancy limit runs as that limit)
        int best_bpc = 0;
        for (int bpc = 1; bpc <= 8 && st == PM_OK; ++bpc) {
            c->bpc = bpc;
            double ms = 0.0;
            st = probe_ms(c, p, u, obs, n_obs, kappa, T, dt, np, seed, tmp, &ms);
            if (st == PM_OK && ms < best) {
                best = ms;
                best_bpc = bpc;
            }
        }
        c->bpc = save_bpc;
        (void)hipFree(tmp);
        if (st) return st;
        c->tune_bpc_mx[p->K] = best_bpc;
        if (bpc_out) *bpc_out = best_bpc;
        if (ms_out) *ms_out = best;
        return PM_OK;
    }
    // the vector kernel: particles per lane and coefficient source
    int best_ppl = 2, best_src = PM_COEF_LDS;
    const int ppls[4] = {1, 2, 3, 4};
    for (int src = 0; src < 2 && st == PM_OK; ++src) {
        for (int pi = 0; pi < 4 && st == PM_OK; ++pi) {
            c->ppl = ppls[pi];
            c->src = src;
            double ms = 0.0;
            st = probe_ms(c, p, u, obs, n_obs, kappa, T, dt, np, seed, tmp, &ms);
            if (st == PM_OK && ms < best) {
                best = ms;
                best_ppl = ppls[pi];
                best_src = src;
            }
        }
    }
    c->ppl = save_ppl;
    c->src = save_src;
    (void)hipFree(tmp);
    if (st) return st;
    c->tune_ppl[p->K] = best_ppl;
    c->tune_src[p->K] = best_src;
    if (ppl_out) *ppl_out = best_ppl;
    if (src_out) *src_out = best_src;
    if (ms_out) *ms_out = best;
    return PM_OK;
}

}  // extern "C"
