// pm_walk.h -- the walk of Algorithm 2, shared by the vector-unit kernel
// (pm_kernels.hip) and the matrix-core kernel (pm_mx.hip); each passes its own
// velocity evaluation.
#pragma once

#include "pm_kernels.h"

namespace pm {

// ---------------------------------------------------------------------------
// Algorithm 2 on the unit disk or square, persistent lanes.
// Each lane walks one particle at a time; a lane whose particle has left the
// disk takes the next particle index from a device queue (one atomic per wave
// per refill).  Refills happen only at even step counts so that all lanes of
// a wave consume the two normal pairs of one Philox block together.
// FK = 0: source f = p0 x + p1 y + p2 (zero, constant, linear) inline;
// FK = 1: any field kind; FK = 2: Gaussian sources, one integral each.
// ---------------------------------------------------------------------------
template <int FK>
__device__ __forceinline__ double source_at(const FieldArg &f, double x, double y)
{
    if constexpr (FK == 0) return __builtin_fma(f.p[0], x, __builtin_fma(f.p[1], y, f.p[2]));
    else return field_eval(f, x, y);
}

// The walk itself: every lane of the block runs it; velocity(x, y, vx, vy)
// is called by all lanes of a wave together at every step (lanes without a
// particle pass their last position), so it may use cross-lane operations.
// C is the particle coordinate (set, at, value, advance, save, load) and sc
// the step constants in its units.
template <typename T, int FK, int DOM, typename C, typename Vel>
__device__ __forceinline__ void dirichlet_walk(const DirArgs<T> &a, const StepConsts<T> &sc, Vel &&velocity)
{
    const int lane = threadIdx.x & 63;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    bool has = false, done = false;
    C x, y;
    x.set(0.0);
    y.set(0.0);
    double I = 0.0;
    double Is[FK == 2 ? PM_MAX_SOURCES : 1];  // per-source integrals (FK = 2)
#pragma unroll
    for (int q = 0; q < (FK == 2 ? PM_MAX_SOURCES : 1); ++q) Is[q] = 0.0;
    int64_t n = 0, t = 0;
    uint32_t pi = 0, pj = 0;

    auto finish = [&](double ex, double ey, bool exited) {
        write_exit_record(a.rec, t, ex, ey, I, n, exited);
        if constexpr (FK == 2) {
#pragma unroll
            for (int q = 0; q < PM_MAX_SOURCES; ++q)
                if (q < a.n_src) a.integ_src[q * a.total + t] = Is[q];
        }
        has = false;
    };

    auto substep = [&](T z0, T z1) {
        T vx, vy;
        velocity(x.at(), y.at(), vx, vy);
        C nx = x, ny = y;
        nx.advance(vx + a.v0x, z0, sc);
        ny.advance(vy + a.v0y, z1, sc);
        if (has) {
            if constexpr (FK == 2) {  // left point, one integral per Gaussian source
                const double xd = x.value(), yd = y.value();
#pragma unroll
                for (int q = 0; q < PM_MAX_SOURCES; ++q) {
                    if (q < a.n_src) {
                        const double dx = xd - a.src[q][0], dy = yd - a.src[q][1];
                        Is[q] += exp(-a.src[q][2] * (dx * dx + dy * dy)) * a.dtd;
                    }
                }
            } else {
                // left point; a constant source (p0 = p1 = 0, wave-uniform)
                // adds p2 dt without the coordinates, bitwise the same value
                if (FK == 0 && a.f.p[0] == 0.0 && a.f.p[1] == 0.0) I += a.f.p[2] * a.dtd;
                else I += source_at<FK>(a.f, x.value(), y.value()) * a.dtd;
            }
            n += 1;
            // The exit test is decided in FP64.  FP32 particles first try the
            // FP32 position: inside by more than 2^-18 (far above the 2^-21
            // that the dropped low part and FP32 rounding can move the test),
            // the FP64 test would say inside too, so it is skipped.
            bool check = true;
            if constexpr (std::is_same<T, float>::value) {
                constexpr float m = 0x1p-18f;
                const float hx = nx.at(), hy = ny.at();
                if constexpr (DOM == PM_DISK) check = !(__builtin_fmaf(hx, hx, hy * hy) < 1.f - m);
                else check = !(hx > m && hx < 1.f - m && hy > m && hy < 1.f - m);
            }
            bool out = false;
            double nxd = 0.0, nyd = 0.0;
            if (check) {
                nxd = nx.value();
                nyd = ny.value();
                if constexpr (DOM == PM_DISK) out = nxd * nxd + nyd * nyd >= 1.0;
                else out = !(nxd > 0.0 && nxd < 1.0 && nyd > 0.0 && nyd < 1.0);
            }
            if (out) {
                // exit point: the nearest boundary point (radial projection
                // onto the circle; clamping onto the square)
                if constexpr (DOM == PM_DISK) {
                    const double r = sqrt(nxd * nxd + nyd * nyd);
                    finish(nxd / r, nyd / r, true);
                } else {
                    finish(fmin(fmax(nxd, 0.0), 1.0), fmin(fmax(nyd, 0.0), 1.0), true);
                }
            } else if (n >= a.max_steps) {
                finish(nx.value(), ny.value(), false);
            } else {
                x = nx;
                y = ny;
            }
        }
    };

    // input: fresh particles (mode 0) or saved walkers (mode 1)
    unsigned long long *const qhead = a.mode ? a.pin.head : a.queue;
    int64_t limit = a.total;
    if (a.mode) {
        limit = (int64_t)uniform64((int64_t)*a.pin.count);
        limit = limit < a.pin.cap ? limit : a.pin.cap;  // hand-overs past a full pool were not stored
    }
    int iters = 0;
    auto save = [&](double *S, int64_t slot) {
        x.save(S[0], S[1]);
        y.save(S[2], S[3]);
        S[4] = I;
        S[5] = (double)n;
        if constexpr (FK == 2) {
#pragma unroll
            for (int q = 0; q < PM_MAX_SOURCES; ++q) S[6 + q] = Is[q];
        }
        a.pout.ij[2 * slot] = pi;
        a.pout.ij[2 * slot + 1] = pj;
    };
    for (;;) {
        if (a.hand_steps > 0) {  // step counts are even here
            const bool give = has && n >= a.hand_steps;
            const unsigned long long gm = __ballot(give);
            if (gm) {
                const int first = __ffsll((long long)gm) - 1;
                unsigned long long base = 0;
                if (lane == first) base = atomicAdd(a.pout.count, (unsigned long long)__popcll(gm));
                base = __shfl(base, first);
                if (give) {
                    const int64_t slot = (int64_t)base + __popcll(gm & ((1ull << lane) - 1ull));
                    if (slot < a.pout.cap) {  // else the pool is full: keep walking here
                        save(a.pout.st + slot * DIR_POOL_WORDS, slot);
                        has = false;
                    }
                }
            }
        }
        const bool need = !has && !done;
        const unsigned long long m = __ballot(need);
        if (m) {
            const int first = __ffsll((long long)m) - 1;
            unsigned long long base = 0;
            if (lane == first) base = atomicAdd(qhead, (unsigned long long)__popcll(m));
            base = __shfl(base, first);
            if (need) {
                const int rank = __popcll(m & ((1ull << lane) - 1ull));
                const int64_t tt = (int64_t)base + rank;
                if (tt < limit) {
                    if (a.mode == 0) {
                        const int64_t jq = tt / a.np;
                        pj = (uint32_t)a.order[jq];
                        pi = (uint32_t)(tt - jq * a.np);
                        x.set(a.obs[2 * pj]);
                        y.set(a.obs[2 * pj + 1]);
                        I = 0.0;
#pragma unroll
                        for (int q = 0; q < (FK == 2 ? PM_MAX_SOURCES : 1); ++q) Is[q] = 0.0;
                        n = 0;
                    } else {  // resume a saved walker where it stopped (an even step count)
                        const double *S = a.pin.st + tt * DIR_POOL_WORDS;
                        x.load(S[0], S[1]);
                        y.load(S[2], S[3]);
                        I = S[4];
                        n = (int64_t)S[5];
                        if constexpr (FK == 2) {
#pragma unroll
                            for (int q = 0; q < PM_MAX_SOURCES; ++q) Is[q] = S[6 + q];
                        }
                        pi = a.pin.ij[2 * tt];
                        pj = a.pin.ij[2 * tt + 1];
                    }
                    t = (int64_t)pj * a.np + pi;
                    has = true;
                } else {
                    done = true;
                }
            }
        }
        const unsigned long long hm = __ballot(has);
        if (hm == 0) break;
        // compaction: the input is exhausted for this wave and too few lanes
        // are still walking; hand the walkers to the next launch
        if (a.dump_below > 0 && iters >= a.min_iters && __ballot(done) != 0 &&
            __popcll(hm) < a.dump_below) {
            const int first = __ffsll((long long)hm) - 1;
            unsigned long long base = 0;
            if (lane == first) base = atomicAdd(a.pout.count, (unsigned long long)__popcll(hm));
            base = __shfl(base, first);
            if (has) {
                const int64_t slot = (int64_t)base + __popcll(hm & ((1ull << lane) - 1ull));
                if (slot < a.pout.cap) {
                    save(a.pout.st + slot * DIR_POOL_WORDS, slot);
                    has = false;
                }
            }
            // a full pool leaves some walkers here: the wave walks on
            if (__ballot(has) == 0) break;
        }
        ++iters;
        const U4 w = philox4x32_10((uint32_t)(n >> 1), pi, pj, 0u, k0, k1);
        T z0, z1, z2, z3;
        C::normals(w.x, w.y, sc, z0, z1);
        C::normals(w.z, w.w, sc, z2, z3);
        substep(z0, z1);
        substep(z2, z3);
    }
}

}  // namespace pm
