/*
 * pm.h -- C ABI of the MI355X (gfx950) particle forward-map library libpm.so.
 *
 * The library evaluates the forward map G(u) = {G_j(u)} of the paper's
 * Problems 2.1 and 2.2 (eq. Gmap) with the particle methods of Section 3:
 * Algorithm 1 (time-dependent advection-diffusion, Theorem 3.1) and
 * Algorithm 2 (Dirichlet boundary-value problem, Theorem 3.2), for the
 * constant-diffusion, divergence-free setting of Section 4.1 (eq. adr,
 * sigma = sqrt(2 kappa) I, velocity of eq. v_expand).
 *
 * Conventions shared by every call
 * --------------------------------
 * - The unknown u is the stream function
 *       psi(x) = sum_m a_m cos(2 pi k_m.x) + b_m sin(2 pi k_m.x),
 *   stored as u = [a_0..a_{M-1}, b_0..b_{M-1}] (FP64) in the order of the
 *   wavevector table given to pm_problem_create; the velocity is
 *       v = (d psi/dy, -d psi/dx) + v0,
 *   which is eq. v_expand with v_k = -pi |k| (b_k + i a_k).  On the unit disk
 *   psi is multiplied by the cutoff (1 - |x|^2)^2 before differentiating.
 * - Particle paths follow eq. (euler) with uniform steps:
 *       X_{n+1} = X_n - v(X_n) dt + sqrt(2 kappa dt) xi_n,
 *   wrapped to [0,1)^2 on the torus.  (Milstein, eq. millstein, is the same
 *   map for constant sigma.)
 * - xi_n comes from Philox4x32-10 (Salmon et al., SC'11) with
 *       key = (seed lo32, seed hi32), counter = (n/2, i, j, 0),
 *   words (w0,w1) for even n and (w2,w3) for odd n, uniforms
 *   ua = ((wa>>8)+1) 2^-24, ub = (wb>>8) 2^-24, and Box-Muller
 *   xi = sqrt(-2 ln ua) (cos 2 pi ub, sin 2 pi ub).  i is the particle index
 *   within observation j, so any path can be replayed from (seed, j, i).
 * - All array arguments marked "device" are device pointers on the context's
 *   device (for example torch tensors' data_ptr()).  Arguments marked "host"
 *   are host pointers read before the call returns.  The caller owns every
 *   buffer; the library owns only the internals of pm_ctx and pm_problem.
 * - Calls enqueue work on the context's stream and return; device results
 *   are valid after pm_sync() (or after synchronising that stream).
 * - Argument errors are detected before any launch and return PM_EINVAL
 *   without side effects.  No call throws across the ABI.
 * - A context is not thread safe: use one per host thread.
 * - FP32 problems keep particle states and the velocity basis in FP32 and
 *   every payoff, exit projection, source integral and mean/variance
 *   accumulation in FP64.
 */
#ifndef PM_H
#define PM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pm_ctx pm_ctx;
typedef struct pm_problem pm_problem;
typedef struct pm_graph pm_graph;

enum pm_status {
    PM_OK = 0,
    PM_EINVAL = -1,       /* bad argument; nothing was launched */
    PM_ENOMEM = -2,       /* device allocation failed */
    PM_EDEVICE = -3,      /* HIP runtime error (launch or sync) */
    PM_ENONFINITE = -4,   /* (pm_sync) a payoff was NaN/Inf */
    PM_ECAPPED = -5,      /* (pm_sync) a Dirichlet path hit max_steps */
    PM_EUNSUPPORTED = -6  /* valid request outside the compiled kernel set */
};

enum pm_domain { PM_TORUS = 0, PM_DISK = 1, PM_SQUARE = 2 };
enum pm_prec { PM_FP32 = 0, PM_FP64 = 1 };

/* Scalar fields theta0 (initial condition), theta_dD (boundary data) and
 * f (source).  params is a host array of n_params doubles (n_params <= 32).
 *   PM_F_ZERO            0
 *   PM_F_CONST           c                                       [c]
 *   PM_F_SINSIN          A sin(2 pi x) sin(2 pi y)               [A]
 *   PM_F_FOURIER         sum c cos 2pi(px+qy) + d sin 2pi(px+qy) [p,q,c,d]*n
 *   PM_F_GAUSS_PERIODIC  sum A sum_{n in {-1,0,1}^2} exp(-|x-c-n|^2/(2 s^2))  [cx,cy,s,A]*n
 *   PM_F_COS_M_THETA     cos(m atan2(y,x))                       [m]
 *   PM_F_EXP_LINEAR      exp(c0 x + c1 y)                        [c0,c1]
 *   PM_F_LINEAR          c0 x + c1 y + c2                        [c0,c1,c2]
 *   PM_F_GAUSS           sum_m A_m exp(-w_m |x - c_m|^2)         [cx,cy,w,A] per term
 *   PM_F_COS_AXES        A (cos(w x) + cos(w y))                 [A, w]
 */
enum pm_field_kind {
    PM_F_ZERO = 0, PM_F_CONST = 1, PM_F_SINSIN = 2, PM_F_FOURIER = 3,
    PM_F_GAUSS_PERIODIC = 4, PM_F_COS_M_THETA = 5, PM_F_EXP_LINEAR = 6, PM_F_LINEAR = 7,
    PM_F_GAUSS = 8, PM_F_COS_AXES = 9
};
#define PM_FIELD_MAX_PARAMS 32

typedef struct {
    int32_t kind;
    int32_t n_params;
    const double *params; /* host */
} pm_field;

/* Largest |k_x|, |k_y| of a wavevector table for the vector-unit kernels
 * (every domain and precision). */
#define PM_MAX_K 8
/* Torus problems in FP32 accept |k_x|, |k_y| up to PM_MAX_K_MFMA: above
 * PM_MAX_K the velocity (eq. v_expand as two bilinear forms in the axis
 * Fourier bases) runs on the matrix cores in split FP16 (hi + lo halves,
 * three products, FP32 accumulation; about FP32 accuracy).  This is the
 * regime of Section 4's turbulent example, |k|_2 <= 80 (20,081 modes). */
#define PM_MAX_K_MFMA 95
/* FP32 torus problems with 1 <= K <= PM_MAX_K_MX (basis entries 0..15 of each
 * axis on the matrix cores, the entry-16 terms of K = 8 on the vector units)
 * and FP32 disk problems with 1 <= K <= PM_MAX_K_DISK_MX
 * run the same bilinear forms on the matrix cores by default (engine
 * PM_ENGINE_AUTO; see pm_set_velocity_engine). */
#define PM_MAX_K_MX 8
#define PM_MAX_K_DISK_MX 4

/* Velocity engines of FP32 problems (pm_set_velocity_engine). */
#define PM_ENGINE_AUTO 0 /* matrix cores where they apply (K <= PM_MAX_K_MX), else vector units */
#define PM_ENGINE_VALU 1 /* vector units: FP32 fused multiply-adds */
#define PM_ENGINE_MFMA 2 /* matrix cores where they apply (the same as AUTO) */

/* Create a context on HIP device `device` that enqueues on `stream`
 * (a hipStream_t; NULL = the null stream).  Returns PM_OK, PM_EINVAL or
 * PM_EDEVICE. */
int pm_create(pm_ctx **out, int device, void *stream);
void pm_destroy(pm_ctx *ctx);
/* Re-bind the context to another stream of the same device. */
int pm_set_stream(pm_ctx *ctx, void *stream);

/* Problem handle: what a chain or an optimiser does not vary.
 *   domain   PM_TORUS (Problem 2.1 on [0,1)^2), PM_SQUARE (Problem 2.2 on
 *            the unit square (0,1)^2, velocity = the periodic Fourier field
 *            of eq. v_expand evaluated on it, plus v0) or PM_DISK (Problem 2.2 on
 *            the unit disk)
 *   n_modes  M >= 0, k: host [M][2] int32 wavevectors, |k_x|,|k_y| <= PM_MAX_K
 *            (<= PM_MAX_K_MFMA for PM_TORUS with PM_FP32; then no wavevector
 *            may be listed twice: PM_EINVAL)
 *   v0       host [2] constant drift added to the Fourier field, or NULL
 *   theta0   host initial condition for pm_observe_time (NULL for PM_DISK)
 *   prec     PM_FP32 or PM_FP64 particle arithmetic
 * The table and theta0 are copied; the caller's arrays may be freed. */
int pm_problem_create(pm_ctx *ctx, pm_problem **out, int domain, int n_modes,
                      const int32_t *k, const double *v0, const pm_field *theta0, int prec);
void pm_problem_destroy(pm_problem *p);

/* Algorithm 1 (Section 3.1): G_j(u) = theta(T, x_j) ~ mean_i theta0(X_T^(i)).
 *   u         device [2M] FP64
 *   obs_pts   device [n_obs][2] FP64 observation points x_j
 *   kappa>=0, T>0, dt>0: N_t = ceil(T/dt) steps of size T/N_t
 *   n_particles >= 1 particles per observation, seed = Philox key
 *   mean, var device [n_obs] FP64: sample mean and unbiased sample variance
 *             of the payoffs theta0(X_T) (standard error = sqrt(var/Np))
 *   endpoints device [n_obs][n_particles][2] FP64 X_T per path, or NULL
 * Requires a PM_TORUS problem with theta0. */
int pm_observe_time(pm_ctx *ctx, const pm_problem *p, const double *u, const double *obs_pts,
                    int n_obs, double kappa, double T, double dt, int64_t n_particles,
                    uint64_t seed, double *mean, double *var, double *endpoints);

/* pm_observe_time without device allocation.  For callers that cannot
 * allocate device memory at call time: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Arguments, results
 * (bitwise those of pm_observe_time: the same kernels, launch sequence and
 * Philox streams), errors and stream semantics are those of pm_observe_time.
 * The call itself calls no hipMalloc, hipFree or other allocating routine:
 * its per-call device buffers (folded coefficients, matrix-core operands,
 * per-chunk partial statistics, final particle states) are carved from one
 * fixed array of PM_NOALLOC_SCRATCH_MIB MiB of device memory that the
 * library holds on each GPU it runs on, from the first pm_create on that GPU
 * until the process ends (the context's own queue counter and error flags,
 * made by pm_create, are used as usual).
 * Limit: n_obs * ceil(n_particles / 64) <= PM_NOALLOC_MAX_CHUNKS (81,920
 * chunks: 5.24e6 particles, e.g. 49 points x 1e5 particles); larger requests
 * return PM_EINVAL before any launch.
 * Sharing: every call on one GPU uses that GPU's one array, whatever its
 * context.  Calls that overlap in time on one GPU (different streams, host
 * threads or contexts) race and give undefined results; calls ordered on one
 * stream, or separated by pm_sync, are safe.  The array keeps the last call's
 * contents; each call writes every value it reads from it before reading. */
#define PM_NOALLOC_MAX_CHUNKS 81920
#define PM_NOALLOC_SCRATCH_MIB 83
int pm_observe_time_noalloc(pm_ctx *ctx, const pm_problem *p, const double *u, const double *obs_pts,
                            int n_obs, double kappa, double T, double dt, int64_t n_particles,
                            uint64_t seed, double *mean, double *var, double *endpoints);

/* Gaussian sources with unknown weights (the optimal-forcing example of
 * Section 4): for f = sum_q f_q phi_q, phi_q(x) = exp(-w_q |x - c_q|^2),
 * Theorem 3.2 gives theta(x_i) = a_i - sum_q B_qi f_q with
 *   a_i  = E[theta_dD(X_tau)]            (0 for a capped path)
 *   B_qi = E[int_0^tau phi_q(X_t) dt]   (left-point rule),
 * so one particle run, recording one integral per source along each path,
 * gives G(F) = a - B^T F for every F (common random numbers make it exact).
 *   PM_SQUARE problems only (else PM_EUNSUPPORTED); 1 <= n_src <= PM_MAX_SOURCES
 *   sources   host [n_src][3] = (cx, cy, w)
 *   bnd_mean, bnd_var  device [n_obs]: mean and variance of theta_dD(X_tau)
 *   src_mean  device [n_src][n_obs]: B
 *   tau_mean, tau_var, n_capped as for pm_observe_dirichlet
 * The exit rule is that of pm_observe_dirichlet on the square. */
#define PM_MAX_SOURCES 4
int pm_observe_dirichlet_sources(pm_ctx *ctx, const pm_problem *p, const double *u, const pm_field *g,
                                 const double *obs_pts, int n_obs, double kappa, double dt, int64_t n_particles,
                                 uint64_t seed, int64_t max_steps, int n_src, const double *sources,
                                 double *bnd_mean, double *bnd_var, double *src_mean, double *tau_mean,
                                 double *tau_var, int64_t *n_capped);

/* Observations at several times along the same paths.  The data of an
 * inverse problem may observe theta at times t_1 < ... < t_R at each point
 * (Section 2: observations are pairs (t_j, x_j); Example 3 of Section 4 reads
 * 13 times at 2 points).  Algorithm 1 run separately per (t_k, x_j) would
 * launch one ensemble per pair; here one ensemble per point is read out as it
 * passes each t_k.  With the same seed and step the readout at t_k is path for
 * path the ensemble Algorithm 1 draws for T = t_k, so each mean has the same
 * law and standard error; means at different times of one point are
 * correlated (shared paths).
 *   read_steps host [n_read], 1 <= n_read <= PM_MAX_READS, strictly
 *              increasing step counts n_k >= 0; t_k = n_k dt (n_k = 0 reads
 *              theta0 at x_j)
 *   dt > 0     the step size (uniform, no rounding to T)
 *   mean, var  device [n_read][n_obs] FP64
 * Other arguments as for pm_observe_time.  PM_EINVAL for an empty, too long,
 * negative or non-increasing read list. */
#define PM_MAX_READS 64
int pm_observe_time_multi(pm_ctx *ctx, const pm_problem *p, const double *u, const double *obs_pts,
                          int n_obs, const int64_t *read_steps, int n_read, double kappa, double dt,
                          int64_t n_particles, uint64_t seed, double *mean, double *var);

/* Replay of one path of Algorithm 1 (eq. euler): the positions X_0 .. X_{N_t}
 * of particle i of observation j in the forward map
 *   pm_observe_time(ctx, p, u, obs_pts, n_obs, kappa, T, dt, n_particles, seed, ...)
 * on the same velocity engine, precision and step size T/N_t, N_t = ceil(T/dt).
 * The path is re-run from x_j by the kernels of that map (with the Philox
 * stream (seed, j, i)), carrying their own particle state (FP64; FP32 hi + lo
 * pair; the matrix-core engine's 32-bit fixed-point fraction of the period),
 * so path[N_t] equals that map's endpoints[j][i] bit for bit and every
 * earlier row is the state the map held after that many steps.
 *   j          0 <= j < n_obs, i: 0 <= i < n_particles
 *   path       device [N_t + 1][2] FP64, each position wrapped to [0,1)^2
 * Other arguments as for pm_observe_time (a PM_TORUS problem with theta0);
 * N_t < PM_REPLAY_MAX_STEPS, else PM_EINVAL.  One wave of 64 particles runs
 * N_t steps, so the call takes roughly the latency of N_t steps. */
#define PM_REPLAY_MAX_STEPS (1 << 30)
int pm_replay_path(pm_ctx *ctx, const pm_problem *p, const double *u, const double *obs_pts, int n_obs,
                   double kappa, double T, double dt, int64_t n_particles, uint64_t seed, int j, int64_t i,
                   double *path);

/* Algorithm 2 (Section 3.2, Theorem 3.2) on the unit disk or the unit square:
 *   payoff_i = theta_dD(X_tau) - int_0^tau f(X_t) dt
 * with the exit detected after a step when Y is no longer inside (disk:
 * |Y|^2 >= 1; square: a coordinate <= 0 or >= 1; tested in FP64), the exit
 * point the nearest boundary point (disk: radial projection; square: Y
 * clamped to [0,1]^2; FP64), tau = n dt for the first outside step n and the
 * source integrated by the left-point rule in FP64.  A path still inside after max_steps steps is capped: its payoff is
 * -int f (no boundary term), it is counted in n_capped and pm_sync() returns
 * PM_ECAPPED.
 *   f, g      host field descriptors (source and boundary data)
 *   mean,var  device [n_obs] payoff statistics
 *   tau_mean, tau_var device [n_obs] exit-time statistics (time units)
 *   n_capped  device [n_obs] int64
 *   paths     device [n_obs][n_particles][4] FP64 (exit x, exit y, payoff,
 *             exit step) per path, or NULL
 * On the disk with FP32 and the matrix-core engine the observation points
 * must have |x|, |y| < 1.5 (see pm_sync). */
int pm_observe_dirichlet(pm_ctx *ctx, const pm_problem *p, const double *u, const pm_field *f,
                         const pm_field *g, const double *obs_pts, int n_obs, double kappa,
                         double dt, int64_t n_particles, uint64_t seed, int64_t max_steps,
                         double *mean, double *var, double *tau_mean, double *tau_var,
                         int64_t *n_capped, double *paths);

/* Many parameter sets in one persistent launch (the same G of Algorithm 1 for
 * each u_b, each with its own particle count and seed).  Results are bitwise
 * equal to n_u separate pm_observe_time calls with the same arguments.
 *   u            device [n_u][2M] FP64
 *   n_particles  host [n_u] int64 (>= 1), seeds host [n_u]
 *   mean, var    device [n_u][n_obs] FP64 */
int pm_observe_time_batch(pm_ctx *ctx, const pm_problem *p, int n_u, const double *u,
                          const int64_t *n_particles, const uint64_t *seeds,
                          const double *obs_pts, int n_obs, double kappa, double T, double dt,
                          double *mean, double *var);

/* Finite-difference Jacobian of the time-problem map G (Algorithm 1):
 *   J[j][k] = (G_j(u + h e_k) - G_j(u - h e_k)) / ((u_k + h) - (u_k - h)),
 * the derivative of G with respect to each of the 2M coefficients, for
 * gradient-based optimisation or samplers (the paper's methods need it from
 * repeated forward maps, its G having no adjoint).  All 4M perturbed maps run
 * in one batched launch with common random numbers (one seed and particle
 * count for every set), so G is a smooth function of u and the differences
 * carry no independent Monte Carlo noise.
 *   u device [2M] FP64, obs_pts device [n_obs][2], h > 0 (coefficient units)
 *   J device [n_obs][2M] FP64
 * Other arguments as for pm_observe_time.  Workspace: 4M x 2M doubles for the
 * perturbed sets plus the batch's own. */
int pm_jacobian_time(pm_ctx *ctx, const pm_problem *p, const double *u, const double *obs_pts, int n_obs,
                     double kappa, double T, double dt, int64_t n_particles, uint64_t seed, double h, double *J);

/* One Euler-Maruyama step per entry (eq. euler), for replaying or checking
 * paths: Y[e] = step n[e] of particle (i[e], j[e]) applied to X[e], in the
 * problem's precision (X is rounded to it first; on the FP32 disk with the
 * matrix-core engine to its 2^-30 fixed-point grid, which requires
 * |x|, |y| < 1.5: other points are reported by pm_sync).
 * Device arrays:
 *   X, Y [count][2] FP64, n [count] uint64, i, j [count] uint32. */
int pm_step(pm_ctx *ctx, const pm_problem *p, const double *u, int64_t count, const double *X,
            const uint64_t *n, const uint32_t *i, const uint32_t *j, double kappa, double dt,
            uint64_t seed, double *Y);

/* Velocity v(X) (eq. v_expand plus v0, with the disk cutoff) at count points
 * in the problem's precision.  Device X, V [count][2] FP64. */
int pm_velocity(pm_ctx *ctx, const pm_problem *p, const double *u, int64_t count,
                const double *X, double *V);

/* Normal pairs xi_n of particle (i, j) in the problem's precision.  Device
 * n [count] uint64, i, j [count] uint32, Z [count][2] FP64. */
int pm_normals(pm_ctx *ctx, const pm_problem *p, int64_t count, const uint64_t *n,
               const uint32_t *i, const uint32_t *j, uint64_t seed, double *Z);

/* Wait for the context's stream.  Returns PM_EDEVICE on a runtime error,
 * else PM_EUNSUPPORTED if a call since the previous pm_sync gave an FP32 disk
 * problem on the matrix-core engine a start point (observation point, or
 * pm_step input) with |x| or |y| >= 1.5, which its fixed-point coordinates
 * do not hold (that call's results are undefined; the vector engine,
 * pm_set_velocity_engine(PM_ENGINE_VALU), takes any point), else
 * PM_ENONFINITE / PM_ECAPPED if a call saw a non-finite payoff or a capped
 * path, else PM_OK.  Clears the flags. */
int pm_sync(pm_ctx *ctx);

/* Time of the last kernel of the most recent observe call, measured with
 * HIP events on the context's stream (milliseconds), and the number of
 * particle-steps it executed.  Valid after pm_sync(). */
int pm_last_kernel_stats(pm_ctx *ctx, double *ms, double *particle_steps);

const char *pm_strerror(int status);

/* Kernel tuning knob for the vector time kernel: particles per lane (1 to 4) and
 * coefficient source (0 = LDS, 1 = scalar cache).  particles_per_lane = 0
 * selects the autotuned choice for the problem's K, else 2 particles per lane.
 * Every choice gives bitwise identical results. */
int pm_set_tuning(pm_ctx *ctx, int particles_per_lane, int coef_source);

/* Velocity engine (eq. v_expand) of FP32 problems:
 *   PM_ENGINE_AUTO (default) or PM_ENGINE_MFMA: on the torus with
 *     1 <= K <= PM_MAX_K_MX (Algorithm 1: pm_observe_time, _multi, _batch,
 *     pm_jacobian_time, the graphs) and on the disk with 1 <= K <= PM_MAX_K_DISK_MX
 *     (Algorithm 2: pm_observe_dirichlet), and in pm_step / pm_velocity for
 *     both, the bilinear forms of 64 particles are one matrix-core
 *     contraction (v_mfma_f32_32x32x16_f16 on coefficients and x basis
 *     split into FP16 hi + lo halves, three products, FP32 accumulation:
 *     velocity errors near 1e-6 of max |v|, paths within the FP32 error
 *     contract);
 *   PM_ENGINE_VALU: FP32 fused multiply-adds on the vector units (the
 *     kernel whose variants pm_set_tuning selects).
 * The matrix-core kernels keep particle coordinates as 32-bit fixed-point
 * numbers: on the torus fractions of the period (resolution 2^-32, the wrap
 * by modular overflow), on the disk multiples of 2^-30 with each step's
 * increment clamped to 1/2 per axis (pm_step on the disk then takes points
 * with |x|, |y| < 1.5, as every walker is; pm_velocity any finite point).  They apply when sqrt(2 kappa dt) <=
 * 0.05; larger steps run on the vector units.  The two engines round differently, so their results agree
 * to that contract, not bit for bit; each is deterministic.  FP64 problems,
 * the square and larger K ignore the setting.  Returns PM_EINVAL for another
 * value or a closed context. */
int pm_set_velocity_engine(pm_ctx *ctx, int engine);

/* Coefficient source of the Dirichlet walk: 0 = LDS, 1 = scalar cache
 * (default).  Both give bitwise identical results. */
int pm_set_dirichlet_source(pm_ctx *ctx, int coef_source);

/* Number of persistent 256-thread blocks per compute unit for the time kernel
 * (0 = as many as occupancy allows). */
int pm_set_blocks_per_cu(pm_ctx *ctx, int blocks_per_cu);

/* The same for the Dirichlet walk (default 2).  Exit times are heavy-tailed,
 * so fewer resident lanes (each walking more particles from the queue) finish
 * sooner than a full chip of lanes with one or two particles each.  Results
 * do not depend on it. */
int pm_set_dirichlet_blocks_per_cu(pm_ctx *ctx, int blocks_per_cu);

/* Compaction of the Dirichlet walk's tail (default off: dump_below 0,
 * launches 8).  Exit times are heavy-tailed, so the last walks run in waves
 * with few live lanes.  Once no fresh particle is left, a wave whose live
 * lanes drop below dump_below (and that has run at least 2,048 steps in its
 * launch) saves its walkers to a pool and ends; up to `launches` follow-up
 * launches deal the pool densely, the last running every walker to its exit.
 * Paths, results and their order are unchanged bit for bit.  On the disk
 * workload the tail is bound by the longest walks' own step latency, not by
 * sparse waves, so this measured no faster there; it is kept for workloads
 * whose tails are wide rather than long. */
int pm_set_dirichlet_compaction(pm_ctx *ctx, int dump_below, int launches);

/* Cooperative tail of the matrix-core disk walk (Algorithm 2 on the unit
 * disk, FP32, K <= 4, zero, constant or linear source; other paths ignore
 * it).  Walkers leave the matrix-core walk for a pool in two ways: once no
 * fresh particle is left, a wave whose live lanes drop below live_below
 * (after 1,024 iterations in its launch) saves all its walkers and ends;
 * and (hand_steps > 0) every walker that has taken hand_steps steps is
 * saved as soon as it reaches them, its lane taking the next particle.  One
 * more launch then runs every saved walker to its exit, one walker per
 * wave: the 64 lanes share each step (lane 16 f + j forms column j of
 * velocity form f, a row-wise sum adds them; one Philox draw per lane gives
 * the normals of 128 steps), so a long walk advances several times faster
 * than alone in a wave of the matrix-core walk.  Same walk, random numbers,
 * update, exit rule and cap; the velocity is summed in another order than
 * the matrix-core contraction, so a continued path differs from an
 * uninterrupted one in rounding, within the same FP32 bounds.  Hand-over by
 * step count depends on each walker's own steps only, so results are
 * bitwise reproducible from call to call; hand-over of sparse waves depends
 * on which walkers share a wave when the queue runs dry, so results may
 * differ between calls in the rounding of the continued paths.  Walkers
 * beyond the pool's room (resident lanes of the launch) stay in the walk.
 * live_below in 0..64, hand_steps >= 0 and even (0, 0: off; default 8, 0).
 * While on, the compaction setting does not apply to this path.  PM_EINVAL
 * outside those ranges. */
int pm_set_dirichlet_tail(pm_ctx *ctx, int live_below, int64_t hand_steps);

/* Walkers the last Dirichlet call on ctx handed to the cooperative tail
 * (0 when the tail did not run).  Synchronises the context's stream. */
int pm_dirichlet_tail_walkers(pm_ctx *ctx, int64_t *walkers);

/* Autotuner for the time kernel (Algorithm 1) of an FP32 problem: times each
 * variant of the kernel the context would run for it on a probe of
 * n_probe_steps steps with the given particle count and stores the fastest
 * for this problem's K in the context.
 *   vector engine: every particles-per-lane (1-4) and coefficient-source
 *     variant (used whenever pm_set_tuning's particles_per_lane is 0);
 *   matrix-core engine (K <= PM_MAX_K_MX): the persistent grid's blocks per
 *     compute unit, 1-8 (used whenever pm_set_blocks_per_cu is 0; a value at
 *     or above the occupancy limit runs as that limit).
 * Results are bitwise identical for every variant, so tuning never changes
 * G(u).  FP64 and high-K problems have one variant (nothing is timed).
 * Synchronous.  Outputs (host, nullable): particles per lane, coefficient
 * source, blocks per compute unit (0 = occupancy limit) and the probe time in
 * milliseconds. */
int pm_autotune_time(pm_ctx *ctx, const pm_problem *p, const double *u, const double *obs_pts,
                     int n_obs, double kappa, double dt, int64_t n_particles, uint64_t seed,
                     int n_probe_steps, int *particles_per_lane, int *coef_source, int *blocks_per_cu,
                     double *probe_ms);

/* Captured forward map.  Records the whole of one pm_observe_time_batch call
 * (coefficient fold, persistent time kernel, payoff/chunk reduction and
 * finalize; n_u = 1 is the single forward map) as a HIP graph with fixed
 * arguments and a private workspace.  pm_graph_launch replays it on the
 * context's current stream; every replay re-reads u and the observation
 * points from the same device buffers, so an MCMC loop writes each proposal
 * into u and replays (Section 4.1 runs long pCN chains of forward maps).
 * Creation runs the map once eagerly (to size the workspace), then captures;
 * it synchronises.  The graph keeps its context and problem alive; destroy
 * it with pm_graph_destroy.  Replays report non-finite results through
 * pm_sync(ctx).  Argument meaning as for pm_observe_time_batch. */
int pm_graph_create_time(pm_ctx *ctx, const pm_problem *p, int n_u, const double *u,
                         const int64_t *n_particles, const uint64_t *seeds, const double *obs_pts,
                         int n_obs, double kappa, double T, double dt, double *mean, double *var,
                         pm_graph **out);
int pm_graph_launch(pm_graph *g);
/* Particle-steps one replay executes. */
int pm_graph_particle_steps(const pm_graph *g, double *steps);
void pm_graph_destroy(pm_graph *g);

#ifdef __cplusplus
}
#endif

#endif /* PM_H */
