// pm_kernels.hip -- gfx950 kernels of the particle forward map.
//
//   k_fold         u -> per-parameter-set coefficient matrices of the velocity
//                  bilinear forms (Section 4.1, eq. v_expand)
//   k_time         Algorithm 1: Euler-Maruyama paths (eq. euler) to time T;
//                  persistent waves pull work from a device queue, so one
//                  launch serves one or many parameter sets
//   k_time_payoff  payoff theta0(X_T) and per-64-particle-chunk mean/variance
//                  by a wave64 shuffle reduction
//   k_dirichlet    Algorithm 2 on the unit disk: each lane walks one particle
//                  until it leaves the disk, then refills from a device queue
//   k_dir_payoff   boundary value minus source integral per particle
//   k_chunk_reduce per-chunk mean/variance of per-particle values
//   k_finalize     per-observation combination of the chunk partials in a
//                  fixed order with compensated sums
//   k_step, k_velocity, k_normals   replay / inspection hooks
#include "pm_kernels.h"
#include "pm_walk.h"

namespace pm {

// ---------------------------------------------------------------------------
// Coefficient folding.
// psi = sum_m a_m cos(2pi k_m.x) + b_m sin(2pi k_m.x) expands, by the
// addition theorems, into products phi_i(x) phi_j(y) of the axis bases
// (phi_0 = 1, phi_{2n-1} = cos 2 pi n s, phi_{2n} = sin 2 pi n s):
//   cos(A+B) = cos A cos B - sin A sin B,  sin(A+B) = sin A cos B + cos A sin B,
// with sin(2pi(-n)s) = -sin(2 pi n s).  The derivative of an axis basis stays
// in the basis: d/ds phi_{2n-1} = -2 pi n phi_{2n}, d/ds phi_{2n} = 2 pi n phi_{2n-1}.
// One block per parameter set; one thread per Psi entry scans the modes in
// order, so the fold is deterministic.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_fold(FoldArgs a, T *__restrict__ coef)
{
    extern __shared__ double psi[];  // [B][B], psi[i*B + j]
    const int B = 2 * a.K + 1;
    const int b = blockIdx.x;
    const double *__restrict__ u = a.u + (int64_t)b * a.u_stride;
    const int M = a.n_modes;
    for (int e = threadIdx.x; e < B * B; e += blockDim.x) {
        const int i = e / B, j = e % B;
        double acc = 0.0;
        for (int m = 0; m < M; ++m) {
            const int kx = a.k[2 * m], ky = a.k[2 * m + 1];
            const int px = kx < 0 ? -kx : kx, py = ky < 0 ? -ky : ky;
            const double sx = kx < 0 ? -1.0 : 1.0, sy = ky < 0 ? -1.0 : 1.0;
            const int cxi = px ? 2 * px - 1 : 0, cyi = py ? 2 * py - 1 : 0;
            const int sxi = 2 * px, syi = 2 * py;
            const double am = u[m], bm = u[M + m];
            if (i == cxi && j == cyi) acc += am;
            if (px && py && i == sxi && j == syi) acc -= sx * sy * am;
            if (px && i == sxi && j == cyi) acc += sx * bm;
            if (py && i == cxi && j == syi) acc += sy * bm;
        }
        psi[e] = acc;
    }
    __syncthreads();
    const int nf = a.domain == PM_DISK ? 3 : 2;  // the square uses the torus field
    const int R = a.row_stride;
    T *__restrict__ out = coef + (int64_t)b * a.coef_stride;
    const double tp = 6.283185307179586476925286766559;
    for (int e = threadIdx.x; e < B * R; e += blockDim.x) {
        const int j = e / R, q = e % R;
        const int i = q / nf, f = q % nf;
        double val = 0.0;
        if (i < B) {
            // Dy[i][j]: coefficient of phi_i(x) phi_j(y) in d psi/dy
            double dy = 0.0, dx = 0.0;
            if (j > 0) {
                const int n = (j + 1) / 2;
                dy = (j & 1) ? tp * n * psi[i * B + j + 1] : -tp * n * psi[i * B + j - 1];
            }
            if (i > 0) {
                const int n = (i + 1) / 2;
                dx = (i & 1) ? tp * n * psi[(i + 1) * B + j] : -tp * n * psi[(i - 1) * B + j];
            }
            if (nf == 2) {
                val = f == 0 ? dy : -dx;                      // v_x = d psi/dy, v_y = -d psi/dx
            } else {
                val = f == 0 ? psi[i * B + j] : (f == 1 ? dy : -dx);
            }
        }
        out[e] = (T)val;
    }
}

// ---------------------------------------------------------------------------
// Wave-level helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Chunk statistics of the lanes' values: count, sum and the sum of squared
// deviations from the chunk mean (two passes over the same fixed tree).
__device__ __forceinline__ void chunk_stats(bool act, double e, double &cnt, double &s, double &m2)
{
    const double ev = act ? e : 0.0;
    s = wave_sum(ev);
    const int c = __popcll(__ballot(act));
    cnt = (double)c;
    const double mu = c ? s / c : 0.0;
    const double d = act ? e - mu : 0.0;
    m2 = wave_sum(d * d);
}

// ---------------------------------------------------------------------------
// Algorithm 1 (time problem on the torus), persistent.
// A task is PPL consecutive 64-particle chunks of one parameter set; lane l of
// chunk q of observation j runs particle i = 64 q + l.  The particle <-> lane
// map and the reduction tree depend only on (j, i), never on the launch shape,
// so results are bitwise independent of PPL, grid size and batching.
// ---------------------------------------------------------------------------
template <typename T, int K, int PPL, bool SC, bool MT>
__global__ __launch_bounds__(256) void k_time(const TimeArgs<T> a)
{
    constexpr int B = Geo<K>::B;
    constexpr int R = Geo<K>::RT;
    constexpr int NC = B * R;
    __shared__ __align__(16) T lds[SC ? 4 : 4 * NC];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    T *my = lds + (SC ? 0 : wid * NC);
    int cur_b = -1;

    for (;;) {
        unsigned long long tk = 0;
        if (lane == 0) tk = atomicAdd(a.queue, 1ull);
        const int64_t task = uniform64((int64_t)__shfl(tk, 0));
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
            tb = uniform64(a.task_off[b]);
            cb = uniform64(a.chunk_off[b]);
            np = uniform64(a.np_arr[b]);
            seed = (uint64_t)uniform64((int64_t)a.seed_arr[b]);
        }
        const int64_t cpo = (np + 63) >> 6;
        const int64_t nch = cpo * a.n_obs;
        const T *__restrict__ Cg = a.coef + (int64_t)b * a.coef_stride;
        if constexpr (!SC) {
            if (b != cur_b) {
                wave_sync_lds();
                for (int e = lane; e < NC; e += 64) my[e] = Cg[e];
                wave_sync_lds();
                cur_b = b;
            }
        }
        const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);

        Coord<T> x[PPL], y[PPL];
        uint32_t pi[PPL], pj[PPL];
        bool act[PPL], cval[PPL];
        int64_t cix[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int64_t c = (task - tb) * PPL + p;
            cval[p] = c < nch;
            const int64_t cc = cval[p] ? c : 0;
            cix[p] = cc;
            const int64_t j = cc / cpo;
            const int64_t q = cc - j * cpo;
            const int64_t i = q * 64 + lane;
            act[p] = cval[p] && i < np;
            pi[p] = (uint32_t)i + a.rp.i_off;
            pj[p] = (uint32_t)j + a.rp.j_off;
            x[p].set(a.obs[2 * j]);
            y[p].set(a.obs[2 * j + 1]);
        }

        auto step = [&](const T (&z0)[PPL], const T (&z1)[PPL]) {
            T phx[PPL][B], phy[PPL][B];
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                trig_basis<T, K>(x[p].at(), phx[p]);
                trig_basis<T, K>(y[p].at(), phy[p]);
            }
            T vx[PPL], vy[PPL];
            // The coefficients are re-read every step (LDS broadcast or
            // scalar cache); the fence / opaque pointer stops the compiler
            // from hoisting all of them out of the step loop into registers.
            if constexpr (SC) {
                torus_velocity<T, K, PPL>(opaque_sgpr((cptr<T>)Cg), phx, phy, vx, vy);
            } else {
                __asm__ volatile("" ::: "memory");
                torus_velocity<T, K, PPL>((const T *)my, phx, phy, vx, vy);
            }
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                x[p].advance(vx[p] + a.v0x, z0[p], a.sc);
                y[p].advance(vy[p] + a.v0y, z1[p], a.sc);
                x[p].wrap();
                y[p].wrap();
            }
        };

        if constexpr (!MT) {
            int64_t n = 0;
            for (; n + 1 < a.n_steps; n += 2) {
                T z0[PPL], z1[PPL], z2[PPL], z3[PPL];
#pragma unroll
                for (int p = 0; p < PPL; ++p) {
                    const U4 w = philox4x32_10_wu((uint32_t)(n >> 1), pi[p], pj[p], k0, k1);
                    box_muller(w.x, w.y, z0[p], z1[p]);
                    box_muller(w.z, w.w, z2[p], z3[p]);
                }
                step(z0, z1);
                step(z2, z3);
            }
            if (n < a.n_steps) {
                T z0[PPL], z1[PPL];
#pragma unroll
                for (int p = 0; p < PPL; ++p) {
                    const U4 w = philox4x32_10_wu((uint32_t)(n >> 1), pi[p], pj[p], k0, k1);
                    box_muller(w.x, w.y, z0[p], z1[p]);
                }
                step(z0, z1);
            }

            // final states, chunk-major: state[(global chunk) * 64 + lane]
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                if (cval[p]) {
                    double *S = a.states + 2 * ((cb + cix[p]) * 64 + lane);
                    S[0] = x[p].value();
                    S[1] = y[p].value();
                }
            }
        } else {
            // Several readouts: after the step that completes read_at[r]
            // steps the positions go to slot r ([r][global chunk][lane]).  The
            // step count is wave-uniform, so the check is a scalar compare.
            int r = 0;
            const bool rp = replay_on(a.rp);
            int64_t next = rp ? 0 : a.read_at[0];
            auto readout = [&](int64_t done) {
                if (done == next) {
                    if (rp) {
                        if (cval[0] && cix[0] == 0 && lane == a.rp.lane) {
                            a.rp.out[2 * r] = x[0].value();
                            a.rp.out[2 * r + 1] = y[0].value();
                        }
                    } else {
#pragma unroll
                        for (int p = 0; p < PPL; ++p) {
                            if (cval[p]) {
                                double *S = a.states + r * a.read_stride + 2 * ((cb + cix[p]) * 64 + lane);
                                S[0] = x[p].value();
                                S[1] = y[p].value();
                            }
                        }
                    }
                    ++r;
                    next = r < a.n_read ? (rp ? r : a.read_at[r]) : -1;
                }
            };

            readout(0);
            int64_t n = 0;
            for (; n + 1 < a.n_steps; n += 2) {
                T z0[PPL], z1[PPL], z2[PPL], z3[PPL];
#pragma unroll
                for (int p = 0; p < PPL; ++p) {
                    const U4 w = philox4x32_10_wu((uint32_t)(n >> 1), pi[p], pj[p], k0, k1);
                    box_muller(w.x, w.y, z0[p], z1[p]);
                    box_muller(w.z, w.w, z2[p], z3[p]);
                }
                step(z0, z1);
                readout(n + 1);
                step(z2, z3);
                readout(n + 2);
            }
            if (n < a.n_steps) {
                T z0[PPL], z1[PPL];
#pragma unroll
                for (int p = 0; p < PPL; ++p) {
                    const U4 w = philox4x32_10_wu((uint32_t)(n >> 1), pi[p], pj[p], k0, k1);
                    box_muller(w.x, w.y, z0[p], z1[p]);
                }
                step(z0, z1);
                readout(n + 1);
            }
        }
    }
}

// Payoff theta0(X_T) (FP64) of every particle and its chunk statistics.  One
// wave per 64-particle chunk; the lane <-> particle map is that of k_time.
__global__ __launch_bounds__(256) void k_time_payoff(const PayArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t ga = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);  // readout-major chunk
    if (ga >= a.n_read * a.n_chunks) return;
    const int64_t g = ga % a.n_chunks;
    int b = 0;
    int64_t cb = 0, np = a.np0;
    if (a.n_u > 1) {
        int lo = 0, hi = a.n_u - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.chunk_off[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        b = lo;
        cb = a.chunk_off[b];
        np = a.np_arr[b];
    }
    const int64_t cpo = (np + 63) >> 6;
    const int64_t c = g - cb;
    const int64_t j = c / cpo, q = c - j * cpo;
    const int64_t i = q * 64 + lane;
    const bool act = i < np;
    double sx, sy;
    if (a.fix_states) {  // position = X 2^-32 in [-1/2, 1/2)
        const uint2 F = reinterpret_cast<const uint2 *>(a.fix_states)[ga * 64 + lane];
        sx = (double)(int32_t)F.x * 0x1p-32;
        sy = (double)(int32_t)F.y * 0x1p-32;
    } else {
        const double *S = a.states + 2 * (ga * 64 + lane);
        sx = S[0];
        sy = S[1];
    }
    const double xd = sx - floor(sx), yd = sy - floor(sy);
    double e = 0.0;
    if (act) e = field_eval(a.theta0, xd, yd);
    if (a.endpoints && act) {
        double *E = a.endpoints + 2 * (j * np + i);
        E[0] = xd;
        E[1] = yd;
    }
    double cnt, s, m2;
    chunk_stats(act, e, cnt, s, m2);
    if (lane == 0) {
        double *P = a.partials + 3 * ga;
        P[0] = cnt;
        P[1] = s;
        P[2] = m2;
        if (!isfinite(s) || !isfinite(m2)) atomicOr(a.flags, PM_FLAG_NONFINITE);
    }
}

template <typename T, int K, int FK, bool SC, int DOM>
__global__ __launch_bounds__(256) void k_dirichlet(const DirArgs<T> a)
{
    constexpr int B = Geo<K>::B;
    constexpr int R = DOM == PM_DISK ? Geo<K>::RD : Geo<K>::RT;
    constexpr int NC = B * R;
    __shared__ __align__(16) T lds[SC ? 4 : NC];
    if constexpr (!SC) {
        for (int e = threadIdx.x; e < NC; e += blockDim.x) lds[e] = a.coef[e];
        __syncthreads();
    }
    dirichlet_walk<T, FK, DOM, Coord<T>>(a, a.sc, [&](T xa, T ya, T &vx, T &vy) {
        T phx[B], phy[B];
        trig_basis<T, K>(xa, phx);
        trig_basis<T, K>(ya, phy);
        // coefficients re-read every step: scalar cache (SGPR operands) or LDS
        if constexpr (DOM == PM_DISK) {
            if constexpr (SC) {
                disk_velocity<T, K>(opaque_sgpr((cptr<T>)a.coef), phx, phy, xa, ya, vx, vy);
            } else {
                __asm__ volatile("" ::: "memory");
                disk_velocity<T, K>((const T *)lds, phx, phy, xa, ya, vx, vy);
            }
        } else {  // the square: the periodic Fourier field, no cutoff
            const T(&px)[1][B] = reinterpret_cast<const T(&)[1][B]>(phx);
            const T(&py)[1][B] = reinterpret_cast<const T(&)[1][B]>(phy);
            T ax[1], ay[1];
            if constexpr (SC) {
                torus_velocity<T, K, 1>(opaque_sgpr((cptr<T>)a.coef), px, py, ax, ay);
            } else {
                __asm__ volatile("" ::: "memory");
                torus_velocity<T, K, 1>((const T *)lds, px, py, ax, ay);
            }
            vx = ax[0];
            vy = ay[0];
        }
    });
}

// Payoff of Theorem 3.2, theta_dD(X_tau) - int_0^tau f dt (no boundary term
// for a capped path), per particle.
__global__ __launch_bounds__(256) void k_dir_payoff(const DirPayArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.total) return;
    const double4 r = reinterpret_cast<const double4 *>(a.rec)[t];
    const double ex = r.x, ey = r.y;
    const bool capped = r.w < 0.0;
    const double steps = capped ? -r.w - 1.0 : r.w;
    const double pay = (capped ? 0.0 : field_eval(a.g, ex, ey)) - r.z;
    a.pay[t] = pay;
    a.tau[t] = steps * a.dtd;
    a.capped[t] = capped ? 1 : 0;
    if (a.paths) {
        double *P = a.paths + 4 * t;
        P[0] = ex;
        P[1] = ey;
        P[2] = pay;
        P[3] = steps;
    }
    if (capped) atomicOr(a.flags, PM_FLAG_CAPPED);
    if (!isfinite(pay)) atomicOr(a.flags, PM_FLAG_NONFINITE);
}

// ---------------------------------------------------------------------------
// Reductions.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chunk_reduce(const double *__restrict__ vals, int64_t np,
                                                      int64_t n_chunks, int64_t cpo,
                                                      double *__restrict__ partials, unsigned *flags)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= n_chunks) return;
    const int64_t j = c / cpo, q = c - j * cpo;
    const int64_t i = q * 64 + lane;
    const bool act = i < np;
    const double e = act ? vals[j * np + i] : 0.0;
    double cnt, s, m2;
    chunk_stats(act, e, cnt, s, m2);
    if (lane == 0) {
        partials[3 * c] = cnt;
        partials[3 * c + 1] = s;
        partials[3 * c + 2] = m2;
        if (!isfinite(s) || !isfinite(m2)) atomicOr(flags, PM_FLAG_NONFINITE);
    }
}

// Neumaier-compensated accumulator.
struct KSum {
    double s, c;
    __device__ void add(double v)
    {
        const double t = s + v;
        if (fabs(s) >= fabs(v)) c += (s - t) + v;
        else c += (v - t) + s;
        s = t;
    }
    __device__ void merge(const KSum &o)
    {
        add(o.s);
        c += o.c;
    }
    __device__ double value() const { return s + c; }
};

__device__ KSum block_ksum(KSum v, double *sh)
{
    // fixed-order tree over the 256 threads of the block
    sh[2 * threadIdx.x] = v.s;
    sh[2 * threadIdx.x + 1] = v.c;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) {
            KSum a{sh[2 * threadIdx.x], sh[2 * threadIdx.x + 1]};
            KSum b{sh[2 * (threadIdx.x + off)], sh[2 * (threadIdx.x + off) + 1]};
            a.merge(b);
            sh[2 * threadIdx.x] = a.s;
            sh[2 * threadIdx.x + 1] = a.c;
        }
        __syncthreads();
    }
    KSum r{sh[0], sh[1]};
    __syncthreads();
    return r;
}

// One block per (parameter set, observation).  Chunk partials (n_c, S_c, M2_c)
// of the group are combined as
//   N = sum n_c, mean = sum S_c / N,
//   M2 = sum [M2_c + n_c (S_c/n_c - mean)^2],  var = M2 / (N - 1),
// the exact decomposition of the sum of squared deviations, in compensated
// arithmetic and a fixed order.
__global__ __launch_bounds__(256) void k_finalize(FinalArgs a)
{
    __shared__ double sh[512];
    const int g = blockIdx.x;
    const int b = g / a.n_obs, j = g - b * a.n_obs;
    int64_t cpo, base;
    if (a.chunk_off) {
        const int64_t np = a.np_arr[b];
        cpo = (np + 63) >> 6;
        base = a.chunk_off[b] + (int64_t)j * cpo;
    } else {
        cpo = a.cpo;
        base = (int64_t)j * cpo;
    }
    const double *__restrict__ P = a.partials + 3 * base;
    KSum s{0.0, 0.0}, nn{0.0, 0.0};
    for (int64_t c = threadIdx.x; c < cpo; c += blockDim.x) {
        nn.add(P[3 * c]);
        s.add(P[3 * c + 1]);
    }
    const double N = block_ksum(nn, sh).value();
    const double S = block_ksum(s, sh).value();
    const double mean = N > 0 ? S / N : 0.0;
    KSum m2{0.0, 0.0};
    for (int64_t c = threadIdx.x; c < cpo; c += blockDim.x) {
        const double nc = P[3 * c];
        if (nc > 0) {
            const double d = P[3 * c + 1] / nc - mean;
            m2.add(P[3 * c + 2]);
            m2.add(nc * d * d);
        }
    }
    const double M2 = block_ksum(m2, sh).value();
    if (threadIdx.x == 0) {
        const double var = N > 1 ? M2 / (N - 1) : 0.0;
        a.mean[g] = mean;
        a.var[g] = var;
        if (!isfinite(mean) || !isfinite(var)) atomicOr(a.flags, PM_FLAG_NONFINITE);
    }
}

__global__ __launch_bounds__(256) void k_count_capped(const unsigned char *__restrict__ capped,
                                                      int64_t np, int64_t *__restrict__ out)
{
    __shared__ long long sh[256];
    const int j = blockIdx.x;
    long long c = 0;
    for (int64_t i = threadIdx.x; i < np; i += blockDim.x) c += capped[(int64_t)j * np + i];
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = sh[0];
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// Order of the Dirichlet walk's observation points: ascending distance from
// the centre, ties by index (order[rank] = point).  Without flow the expected
// exit time from the unit disk, (1 - |x|^2) / (4 kappa), falls with |x|, so
// the longest walks are dealt first.  One thread per point counts the points
// that precede it.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_walk_order(const double *__restrict__ obs, int n_obs, int domain,
                                                    int *__restrict__ order)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_obs) return;
    // disk: distance from the origin; square: from its centre (1/2, 1/2)
    const double c = domain == PM_DISK ? 0.0 : 0.5;
    // NaN keys count as +inf, so (key, index) is a strict total order and the
    // ranks form a permutation whatever the input holds
    auto key = [&](int q) {
        const double dx = obs[2 * q] - c, dy = obs[2 * q + 1] - c;
        const double k = dx * dx + dy * dy;
        return k == k ? k : __builtin_inf();
    };
    const double ki = key(i);
    int rank = 0;
    for (int q = 0; q < n_obs; ++q) {
        const double kq = key(q);
        rank += (kq < ki || (kq == ki && q < i)) ? 1 : 0;
    }
    order[rank] = i;
}

__global__ void k_pool_reset(unsigned long long *in_head, unsigned long long *out_count)
{
    if (threadIdx.x == 0) {
        *in_head = 0ull;
        *out_count = 0ull;
    }
}

hipError_t launch_pool_reset(unsigned long long *in_head, unsigned long long *out_count, hipStream_t st)
{
    hipLaunchKernelGGL(k_pool_reset, dim3(1), dim3(64), 0, st, in_head, out_count);
    return hipGetLastError();
}

// At most 8 blocks of 256 threads per CU are resident (32 waves per CU).
int64_t dirichlet_max_lanes(int n_cu) { return (int64_t)n_cu * 8 * 256; }

hipError_t launch_walk_order(const double *obs, int n_obs, int domain, int *order, hipStream_t st)
{
    hipLaunchKernelGGL(k_walk_order, dim3((n_obs + 255) / 256), dim3(256), 0, st, obs, n_obs, domain, order);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Finite differences: set 2k is u + h e_k, set 2k+1 is u - h e_k; the
// Jacobian divides the difference of their means by the difference of the
// coefficients actually evaluated (u_k + h) - (u_k - h).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fd_sets(const double *__restrict__ u, int n_coef, double h,
                                                 double *__restrict__ U)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = 2 * (int64_t)n_coef * n_coef;
    if (e >= total) return;
    const int64_t set = e / n_coef;
    const int c = (int)(e - set * n_coef);
    const int k = (int)(set >> 1);
    double v = u[c];
    if (c == k) v = (set & 1) ? v - h : v + h;
    U[e] = v;
}

__global__ __launch_bounds__(256) void k_fd_diff(const double *__restrict__ U, const double *__restrict__ mean,
                                                 int n_obs, int n_coef, double *__restrict__ J)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n_obs * n_coef) return;
    const int j = (int)(e / n_coef), k = (int)(e - (int64_t)j * n_coef);
    const double dk = U[(int64_t)(2 * k) * n_coef + k] - U[(int64_t)(2 * k + 1) * n_coef + k];
    J[e] = (mean[(int64_t)(2 * k) * n_obs + j] - mean[(int64_t)(2 * k + 1) * n_obs + j]) / dk;
}

hipError_t launch_fd_sets(const double *u, int n_coef, double h, double *U, hipStream_t st)
{
    const int64_t total = 2 * (int64_t)n_coef * n_coef;
    hipLaunchKernelGGL(k_fd_sets, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, u, n_coef, h, U);
    return hipGetLastError();
}

hipError_t launch_fd_diff(const double *U, const double *mean, int n_obs, int n_coef, double *J, hipStream_t st)
{
    const int64_t total = (int64_t)n_obs * n_coef;
    hipLaunchKernelGGL(k_fd_diff, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, U, mean, n_obs, n_coef,
                       J);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Replay / inspection hooks (same device functions as the main kernels).
// ---------------------------------------------------------------------------
template <typename T, int K>
__device__ __forceinline__ void velocity_at(const T *__restrict__ C, int domain, T x, T y, T &vx, T &vy)
{
    T phx[2 * K + 1], phy[2 * K + 1];
    trig_basis<T, K>(x, phx);
    trig_basis<T, K>(y, phy);
    if (domain != PM_DISK) {  // torus, and the square (the periodic field evaluated on it)
        const T(&px)[1][2 * K + 1] = reinterpret_cast<const T(&)[1][2 * K + 1]>(phx);
        const T(&py)[1][2 * K + 1] = reinterpret_cast<const T(&)[1][2 * K + 1]>(phy);
        T ax[1], ay[1];
        torus_velocity<T, K, 1>(C, px, py, ax, ay);
        vx = ax[0];
        vy = ay[0];
    } else {
        disk_velocity<T, K>(C, phx, phy, x, y, vx, vy);
    }
}

template <typename T, int K>
__global__ __launch_bounds__(256) void k_step(const StepArgs<T> a)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.count) return;
    Coord<T> x, y;
    x.set(a.X[2 * e]);
    y.set(a.X[2 * e + 1]);
    const uint64_t n = a.n[e];
    const U4 w = philox4x32_10((uint32_t)(n >> 1), a.i[e], a.j[e], 0u, (uint32_t)a.seed,
                               (uint32_t)(a.seed >> 32));
    T z0, z1;
    if ((n & 1) == 0) box_muller(w.x, w.y, z0, z1);
    else box_muller(w.z, w.w, z0, z1);
    T vx, vy;
    velocity_at<T, K>(a.coef, a.domain, x.at(), y.at(), vx, vy);
    x.advance(vx + a.v0x, z0, a.sc);
    y.advance(vy + a.v0y, z1, a.sc);
    double nx = x.value(), ny = y.value();
    if (a.domain == PM_TORUS) {
        nx -= floor(nx);
        ny -= floor(ny);
    }
    a.Y[2 * e] = nx;
    a.Y[2 * e + 1] = ny;
}

template <typename T, int K>
__global__ __launch_bounds__(256) void k_velocity(const T *__restrict__ coef, int domain, T v0x,
                                                  T v0y, int64_t count, const double *__restrict__ X,
                                                  double *__restrict__ V)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    Coord<T> x, y;
    x.set(X[2 * e]);
    y.set(X[2 * e + 1]);
    T vx, vy;
    velocity_at<T, K>(coef, domain, x.at(), y.at(), vx, vy);
    V[2 * e] = (double)(vx + v0x);
    V[2 * e + 1] = (double)(vy + v0y);
}

template <typename T>
__global__ __launch_bounds__(256) void k_normals(int64_t count, const uint64_t *__restrict__ n,
                                                 const uint32_t *__restrict__ i,
                                                 const uint32_t *__restrict__ j, uint64_t seed,
                                                 double *__restrict__ Z)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const uint64_t s = n[e];
    const U4 w = philox4x32_10((uint32_t)(s >> 1), i[e], j[e], 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
    T z0, z1;
    if ((s & 1) == 0) box_muller(w.x, w.y, z0, z1);
    else box_muller(w.z, w.w, z0, z1);
    Z[2 * e] = (double)z0;
    Z[2 * e + 1] = (double)z1;
}

// ---------------------------------------------------------------------------
// Host-side launchers (dispatch over the compile-time harmonic count K).
// ---------------------------------------------------------------------------
template <typename F>
static hipError_t dispatch_k(int K, F &&f)
{
    switch (K) {
    case 0: return f(std::integral_constant<int, 0>{});
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

int row_stride(int domain, int K)
{
    const int B = 2 * K + 1;
    const int nf = domain == PM_DISK ? 3 : 2;
    return ((nf * B + 3) / 4) * 4;
}

template <typename T>
hipError_t launch_fold(const FoldArgs &a, T *coef, int n_sets, hipStream_t st)
{
    const int B = 2 * a.K + 1;
    hipLaunchKernelGGL(k_fold<T>, dim3(n_sets), dim3(256), (size_t)B * B * sizeof(double), st, a, coef);
    return hipGetLastError();
}
template hipError_t launch_fold<float>(const FoldArgs &, float *, int, hipStream_t);
template hipError_t launch_fold<double>(const FoldArgs &, double *, int, hipStream_t);

template <typename T, int K, int PPL, bool SC, bool MT = false>
static hipError_t launch_time_k(const TimeArgs<T> &a, int n_cu, int bpc, hipStream_t st)
{
    auto kern = k_time<T, K, PPL, SC, MT>;
    int per_cu = 0;
    hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0);
    if (err != hipSuccess) return err;
    if (per_cu < 1) per_cu = 1;
    if (bpc > 0 && bpc < per_cu) per_cu = bpc;
    int64_t blocks = (int64_t)per_cu * n_cu;
    const int64_t need = (a.n_tasks + 3) / 4;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_time(const TimeArgs<T> &a, int K, int ppl, int src, int n_cu, int bpc, hipStream_t st)
{
    return dispatch_k(K, [&](auto kc) -> hipError_t {
        constexpr int KK = decltype(kc)::value;
        if (a.n_read > 1) {
            // several readouts: one variant per precision
            if constexpr (std::is_same<T, double>::value) return launch_time_k<T, KK, 1, false, true>(a, n_cu, bpc, st);
            else return launch_time_k<T, KK, 2, true, true>(a, n_cu, bpc, st);
        }
        if constexpr (std::is_same<T, double>::value) {
            return launch_time_k<T, KK, 1, false>(a, n_cu, bpc, st);
        } else {
            if (src == PM_COEF_SCALAR) {
                if (ppl == 1) return launch_time_k<T, KK, 1, true>(a, n_cu, bpc, st);
                if (ppl == 3) return launch_time_k<T, KK, 3, true>(a, n_cu, bpc, st);
                if (ppl == 4) return launch_time_k<T, KK, 4, true>(a, n_cu, bpc, st);
                return launch_time_k<T, KK, 2, true>(a, n_cu, bpc, st);
            }
            if (ppl == 1) return launch_time_k<T, KK, 1, false>(a, n_cu, bpc, st);
            if (ppl == 3) return launch_time_k<T, KK, 3, false>(a, n_cu, bpc, st);
            if (ppl == 4) return launch_time_k<T, KK, 4, false>(a, n_cu, bpc, st);
            return launch_time_k<T, KK, 2, false>(a, n_cu, bpc, st);
        }
    });
}
template hipError_t launch_time<float>(const TimeArgs<float> &, int, int, int, int, int, hipStream_t);
template hipError_t launch_time<double>(const TimeArgs<double> &, int, int, int, int, int, hipStream_t);

template <typename T>
hipError_t launch_dirichlet(const DirArgs<T> &a, int K, int fk, int src, int n_cu, int bpc, int domain,
                            hipStream_t st)
{
    return dispatch_k(K, [&](auto kc) -> hipError_t {
        constexpr int KK = decltype(kc)::value;
        // disk: both coefficient sources; square: scalar cache only, plus the
        // Gaussian-source integrals (fk = 2)
        void (*kern)(const DirArgs<T>);
        if (domain == PM_DISK)
            kern = src == PM_COEF_SCALAR
                       ? (fk == 0 ? k_dirichlet<T, KK, 0, true, PM_DISK> : k_dirichlet<T, KK, 1, true, PM_DISK>)
                       : (fk == 0 ? k_dirichlet<T, KK, 0, false, PM_DISK> : k_dirichlet<T, KK, 1, false, PM_DISK>);
        else
            kern = fk == 0 ? k_dirichlet<T, KK, 0, true, PM_SQUARE>
                           : (fk == 1 ? k_dirichlet<T, KK, 1, true, PM_SQUARE> : k_dirichlet<T, KK, 2, true, PM_SQUARE>);
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
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, st, a);
        return hipGetLastError();
    });
}
template hipError_t launch_dirichlet<float>(const DirArgs<float> &, int, int, int, int, int, int, hipStream_t);
template hipError_t launch_dirichlet<double>(const DirArgs<double> &, int, int, int, int, int, int, hipStream_t);

hipError_t launch_dir_payoff(const DirPayArgs &a, hipStream_t st)
{
    const int64_t blocks = (a.total + 255) / 256;
    hipLaunchKernelGGL(k_dir_payoff, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_time_payoff(const PayArgs &a, hipStream_t st)
{
    const int64_t blocks = (a.n_read * a.n_chunks + 3) / 4;
    hipLaunchKernelGGL(k_time_payoff, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_wrap_path(double *__restrict__ v, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) v[e] -= floor(v[e]);
}

hipError_t launch_wrap_path(double *path, int64_t n_values, hipStream_t st)
{
    if (n_values < 1) return hipSuccess;
    hipLaunchKernelGGL(k_wrap_path, dim3((unsigned)((n_values + 255) / 256)), dim3(256), 0, st, path, n_values);
    return hipGetLastError();
}

hipError_t launch_chunk_reduce(const double *vals, int64_t np, int n_obs, double *partials,
                               unsigned *flags, hipStream_t st)
{
    const int64_t cpo = (np + 63) >> 6;
    const int64_t nch = cpo * n_obs;
    const int64_t blocks = (nch + 3) / 4;
    hipLaunchKernelGGL(k_chunk_reduce, dim3((unsigned)blocks), dim3(256), 0, st, vals, np, nch, cpo,
                       partials, flags);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalArgs &a, int n_groups, hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize, dim3(n_groups), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_count_capped(const unsigned char *capped, int64_t np, int n_obs, int64_t *out,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_count_capped, dim3(n_obs), dim3(256), 0, st, capped, np, out);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_u64, dim3((n + 63) / 64), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step(const StepArgs<T> &a, int K, hipStream_t st)
{
    return dispatch_k(K, [&](auto kc) -> hipError_t {
        constexpr int KK = decltype(kc)::value;
        const int64_t blocks = (a.count + 255) / 256;
        hipLaunchKernelGGL((k_step<T, KK>), dim3((unsigned)blocks), dim3(256), 0, st, a);
        return hipGetLastError();
    });
}
template hipError_t launch_step<float>(const StepArgs<float> &, int, hipStream_t);
template hipError_t launch_step<double>(const StepArgs<double> &, int, hipStream_t);

template <typename T>
hipError_t launch_velocity(const T *coef, int domain, int K, T v0x, T v0y, int64_t count,
                           const double *X, double *V, hipStream_t st)
{
    return dispatch_k(K, [&](auto kc) -> hipError_t {
        constexpr int KK = decltype(kc)::value;
        const int64_t blocks = (count + 255) / 256;
        hipLaunchKernelGGL((k_velocity<T, KK>), dim3((unsigned)blocks), dim3(256), 0, st, coef, domain,
                           v0x, v0y, count, X, V);
        return hipGetLastError();
    });
}
template hipError_t launch_velocity<float>(const float *, int, int, float, float, int64_t, const double *,
                                           double *, hipStream_t);
template hipError_t launch_velocity<double>(const double *, int, int, double, double, int64_t,
                                            const double *, double *, hipStream_t);

template <typename T>
hipError_t launch_normals(int64_t count, const uint64_t *n, const uint32_t *i, const uint32_t *j,
                          uint64_t seed, double *Z, hipStream_t st)
{
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_normals<T>, dim3((unsigned)blocks), dim3(256), 0, st, count, n, i, j, seed, Z);
    return hipGetLastError();
}
template hipError_t launch_normals<float>(int64_t, const uint64_t *, const uint32_t *, const uint32_t *,
                                          uint64_t, double *, hipStream_t);
template hipError_t launch_normals<double>(int64_t, const uint64_t *, const uint32_t *, const uint32_t *,
                                           uint64_t, double *, hipStream_t);

}  // namespace pm
