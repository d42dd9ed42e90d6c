/*
 * pm_oracle.c -- plain FP64 CPU oracle of the particle forward map.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this library.  The HIP
 * library never links it, and it shares no code with the HIP path.
 *
 * It follows the paper step by step, in FP64, with no blocking, fusion or
 * reordering:
 *   - Algorithm 1 (time-dependent problem, Section 3.1): start each particle
 *     at the observation point, advance the Ito diffusion of Theorem 3.1,
 *       dX = -v(X) dt + sigma dW,  X_0 = x_j,
 *     with the Euler-Maruyama map of eq. (euler) for N_t uniform steps to
 *     time T, read theta0 at the end point; G_j is the particle mean.
 *     With constant sigma = sqrt(2 kappa) I (Section 4.1, eq. adr) the
 *     Milstein correction of eq. (millstein) vanishes, so the two schemes
 *     are the same map.
 *   - Algorithm 2 (Dirichlet problem, Section 3.2, Theorem 3.2): step until
 *     the particle leaves the domain, integrating f along the way (left-point
 *     rule), then read the boundary value at the exit point; the payoff is
 *     theta_dD(X_tau) - int_0^tau f(X_t) dt.
 *   - The velocity is the divergence-free Fourier field of eq. (v_expand),
 *     written as v = (d psi/dy, -d psi/dx) for the stream function
 *     psi = sum_k a_k cos(2 pi k.x) + b_k sin(2 pi k.x); every mode is
 *     evaluated with its own libm sin/cos (no recurrences).
 *   - The normals xi of eq. (euler) come from Philox4x32-10 (Salmon, Moraes,
 *     Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) and
 *     the Box-Muller transform (Box and Muller, 1958), under the counter
 *     convention documented at orc_normals.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11 paper): 10 rounds of the Philox S-box on a 4-word   */
/* counter with a 2-word key bumped by the Weyl constants between rounds.   */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/*
 * Normal pair xi_n (2 components) for step n of particle i of observation j.
 *   key     = (seed & 0xffffffff, seed >> 32)
 *   counter = (n / 2, i, j, 0)
 *   words (w0, w1) serve the even step 2*(n/2), (w2, w3) the odd step.
 *   uniforms  ua = ((wa >> 8) + 1) * 2^-24  in (0, 1]
 *             ub =  (wb >> 8)      * 2^-24  in [0, 1)
 *   Box-Muller: r = sqrt(-2 ln ua), xi = (r cos 2 pi ub, r sin 2 pi ub).
 * Both uniforms are exactly representable in FP32 and FP64.
 */
void orc_normals(uint64_t seed, uint64_t n, uint32_t i, uint32_t j, double z[2])
{
    uint32_t ctr[4] = {(uint32_t)(n / 2), i, j, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    uint32_t wa = (n % 2 == 0) ? w[0] : w[2];
    uint32_t wb = (n % 2 == 0) ? w[1] : w[3];
    double ua = ((double)(wa >> 8) + 1.0) * ldexp(1.0, -24);
    double ub = (double)(wb >> 8) * ldexp(1.0, -24);
    double r = sqrt(-2.0 * log(ua));
    z[0] = r * cos(2.0 * M_PI * ub);
    z[1] = r * sin(2.0 * M_PI * ub);
}

/* ------------------------------------------------------------------------ */
/* Scalar fields: initial condition theta0, boundary data and source.       */
/* ------------------------------------------------------------------------ */
enum {
    ORC_F_ZERO = 0,
    ORC_F_CONST = 1,
    ORC_F_SINSIN = 2,
    ORC_F_FOURIER = 3,
    ORC_F_GAUSS_PERIODIC = 4,
    ORC_F_COS_M_THETA = 5,
    ORC_F_EXP_LINEAR = 6,
    ORC_F_LINEAR = 7,
    ORC_F_GAUSS = 8,
    ORC_F_COS_AXES = 9
};

typedef struct {
    int kind;
    int n_params;
    const double *p;
} orc_field;

double orc_field_eval(const orc_field *f, double x, double y)
{
    const double *p = f->p;
    double s = 0.0;
    switch (f->kind) {
    case ORC_F_ZERO:
        return 0.0;
    case ORC_F_CONST:
        return p[0];
    case ORC_F_SINSIN:
        return p[0] * sin(2.0 * M_PI * x) * sin(2.0 * M_PI * y);
    case ORC_F_FOURIER:
        for (int m = 0; m + 3 < f->n_params; m += 4) {
            double ph = 2.0 * M_PI * (p[m] * x + p[m + 1] * y);
            s += p[m + 2] * cos(ph) + p[m + 3] * sin(ph);
        }
        return s;
    case ORC_F_GAUSS_PERIODIC:
        for (int m = 0; m + 3 < f->n_params; m += 4) {
            double cx = p[m], cy = p[m + 1], sg = p[m + 2], A = p[m + 3];
            for (int nx = -1; nx <= 1; ++nx)
                for (int ny = -1; ny <= 1; ++ny) {
                    double dx = x - cx - nx, dy = y - cy - ny;
                    s += A * exp(-(dx * dx + dy * dy) / (2.0 * sg * sg));
                }
        }
        return s;
    case ORC_F_COS_M_THETA:
        return cos(p[0] * atan2(y, x));
    case ORC_F_EXP_LINEAR:
        return exp(p[0] * x + p[1] * y);
    case ORC_F_LINEAR:
        return p[0] * x + p[1] * y + p[2];
    case ORC_F_GAUSS: /* sum_m A_m exp(-w_m |x - c_m|^2), not periodised */
        for (int m = 0; m + 3 < f->n_params; m += 4) {
            double dx = x - p[m], dy = y - p[m + 1];
            s += p[m + 3] * exp(-p[m + 2] * (dx * dx + dy * dy));
        }
        return s;
    case ORC_F_COS_AXES: /* A (cos(w x) + cos(w y)) */
        return p[0] * (cos(p[1] * x) + cos(p[1] * y));
    default:
        return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* Stream function and velocity (Section 4.1, eq. v_expand).                */
/* u = [a_0..a_{M-1}, b_0..b_{M-1}], mode m has wavevector k[2m], k[2m+1].  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int domain;            /* 0 torus [0,1)^2, 1 unit disk, 2 unit square [0,1]^2 (the
                              periodic Fourier field evaluated on it, no cutoff) */
    int n_modes;
    const int32_t *k;      /* [n_modes][2] */
    const double *u;       /* [2 n_modes] */
    double v0[2];          /* constant drift added to the Fourier field */
} orc_flow;

/* Fourier part: psi_F and its gradient, each mode evaluated directly. */
static void fourier_psi(const orc_flow *fl, double x, double y,
                        double *psi, double *dpx, double *dpy)
{
    int M = fl->n_modes;
    double s = 0.0, gx = 0.0, gy = 0.0;
    for (int m = 0; m < M; ++m) {
        double kx = fl->k[2 * m], ky = fl->k[2 * m + 1];
        double a = fl->u[m], b = fl->u[M + m];
        double ph = 2.0 * M_PI * (kx * x + ky * y);
        double c = cos(ph), sn = sin(ph);
        s += a * c + b * sn;
        /* d/dx [a cos + b sin] = 2 pi kx (-a sin + b cos) */
        gx += 2.0 * M_PI * kx * (-a * sn + b * c);
        gy += 2.0 * M_PI * ky * (-a * sn + b * c);
    }
    *psi = s; *dpx = gx; *dpy = gy;
}

/* Stream function: torus psi_F; disk chi * psi_F with cutoff chi = (1-r^2)^2. */
double orc_psi(const orc_flow *fl, double x, double y)
{
    double p, gx, gy;
    fourier_psi(fl, x, y, &p, &gx, &gy);
    if (fl->domain == 1) {
        double w = 1.0 - (x * x + y * y);
        p *= w * w;
    }
    return p;
}

/* v = (d psi/dy, -d psi/dx) + v0. On the disk psi = chi psi_F, so
   grad psi = chi grad psi_F + psi_F grad chi, grad chi = -4 (1 - r^2) x. */
void orc_velocity(const orc_flow *fl, double x, double y, double v[2])
{
    double p, gx, gy;
    fourier_psi(fl, x, y, &p, &gx, &gy);
    if (fl->domain == 1) {
        double w = 1.0 - (x * x + y * y);
        double chi = w * w;
        double cx = -4.0 * w * x, cy = -4.0 * w * y;
        gx = chi * gx + p * cx;
        gy = chi * gy + p * cy;
    }
    v[0] = gy + fl->v0[0];
    v[1] = -gx + fl->v0[1];
}

/* ------------------------------------------------------------------------ */
/* One Euler-Maruyama step, eq. (euler) with sigma = sqrt(2 kappa) I:        */
/*   X_{n+1} = X_n - v(X_n) dt + sqrt(2 kappa dt) xi_n                       */
/* On the torus the result is wrapped to [0,1)^2.                            */
/* ------------------------------------------------------------------------ */
static void em_step(const orc_flow *fl, double kappa, double dt, uint64_t seed,
                    uint64_t n, uint32_t i, uint32_t j, const double X[2], double Y[2])
{
    double v[2], z[2];
    orc_velocity(fl, X[0], X[1], v);
    orc_normals(seed, n, i, j, z);
    double s = sqrt(2.0 * kappa * dt);
    Y[0] = X[0] - v[0] * dt + s * z[0];
    Y[1] = X[1] - v[1] * dt + s * z[1];
    if (fl->domain == 0) {
        Y[0] -= floor(Y[0]);
        Y[1] -= floor(Y[1]);
    }
}

/* Teacher-forced single steps: for each entry e, advance X[e] by step n[e]
   of particle (i[e], j[e]).  Y may alias nothing. */
void orc_step(const orc_flow *fl, double kappa, double dt, uint64_t seed, int64_t count,
              const double *X, const uint64_t *n, const uint32_t *i, const uint32_t *j,
              double *Y)
{
    for (int64_t e = 0; e < count; ++e)
        em_step(fl, kappa, dt, seed, n[e], i[e], j[e], X + 2 * e, Y + 2 * e);
}

/* Number of uniform steps to reach T: N_t = ceil(T/dt) (to 1e-9), dt_eff = T/N_t. */
int64_t orc_n_steps(double T, double dt)
{
    return (int64_t)ceil(T / dt - 1e-9);
}

/* Full path of particle i of observation point x0 (index j): states after
   each of n_steps steps of size dt_eff, out[(n_steps+1)][2] with out[0] = x0. */
void orc_path(const orc_flow *fl, double kappa, double dt_eff, uint64_t seed, uint32_t i,
              uint32_t j, const double x0[2], int64_t n_steps, double *out)
{
    double X[2] = {x0[0], x0[1]};
    out[0] = X[0]; out[1] = X[1];
    for (int64_t n = 0; n < n_steps; ++n) {
        double Y[2];
        em_step(fl, kappa, dt_eff, seed, (uint64_t)n, i, j, X, Y);
        X[0] = Y[0]; X[1] = Y[1];
        out[2 * (n + 1)] = X[0];
        out[2 * (n + 1) + 1] = X[1];
    }
}

/*
 * Algorithm 1.  payoff[j*Np + i] = theta0(X_T) of particle i launched from
 * obs[j]; endpoints (nullable) receive X_T.  The loops over (j, i) are
 * independent (Section 3.3) and run under OpenMP.
 */
void orc_observe_time_steps(const orc_flow *fl, const orc_field *theta0, const double *obs,
                            int n_obs, double kappa, double dte, int64_t Nt, int64_t Np,
                            uint64_t seed, double *payoff, double *endpoints);

void orc_observe_time(const orc_flow *fl, const orc_field *theta0, const double *obs,
                      int n_obs, double kappa, double T, double dt, int64_t Np, uint64_t seed,
                      double *payoff, double *endpoints)
{
    int64_t Nt = orc_n_steps(T, dt);
    orc_observe_time_steps(fl, theta0, obs, n_obs, kappa, T / (double)Nt, Nt, Np, seed, payoff,
                           endpoints);
}

/* Algorithm 1 with Nt steps of the given size dte (Nt = 0 reads theta0 at the
   start points). */
void orc_observe_time_steps(const orc_flow *fl, const orc_field *theta0, const double *obs,
                            int n_obs, double kappa, double dte, int64_t Nt, int64_t Np,
                            uint64_t seed, double *payoff, double *endpoints)
{
    int64_t total = (int64_t)n_obs * Np;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < total; ++t) {
        int64_t j = t / Np, i = t % Np;
        double X[2] = {obs[2 * j], obs[2 * j + 1]};
        for (int64_t n = 0; n < Nt; ++n) {
            double Y[2];
            em_step(fl, kappa, dte, seed, (uint64_t)n, (uint32_t)i, (uint32_t)j, X, Y);
            X[0] = Y[0]; X[1] = Y[1];
        }
        payoff[t] = orc_field_eval(theta0, X[0], X[1]);
        if (endpoints) {
            endpoints[2 * t] = X[0];
            endpoints[2 * t + 1] = X[1];
        }
    }
}

/* Has the step left the domain?  If so, the exit point: the nearest point of
   the boundary (disk: radial projection Y/|Y|; square: Y clamped to
   [0,1]^2, coordinate by coordinate). */
static int left_domain(int domain, const double Y[2], double E[2])
{
    if (domain == 2) {
        if (Y[0] > 0.0 && Y[0] < 1.0 && Y[1] > 0.0 && Y[1] < 1.0) return 0;
        E[0] = Y[0] < 0.0 ? 0.0 : (Y[0] > 1.0 ? 1.0 : Y[0]);
        E[1] = Y[1] < 0.0 ? 0.0 : (Y[1] > 1.0 ? 1.0 : Y[1]);
        return 1;
    }
    double r2 = Y[0] * Y[0] + Y[1] * Y[1];
    if (r2 < 1.0) return 0;
    double r = sqrt(r2);
    E[0] = Y[0] / r;
    E[1] = Y[1] / r;
    return 1;
}

/*
 * Algorithm 2 on the unit disk D = {|x| < 1} or the unit square (0,1)^2.
 *   X = x_j, I = 0, n = 0
 *   repeat:  Y = EM step of X (step index n); I += f(X) dt; n += 1
 *            if Y is not in D: exit point X_tau = the nearest boundary point
 *                              to Y (left_domain), tau = n dt, stop
 *            X = Y; if n == max_steps: the path is capped, stop
 *   payoff = theta_dD(X_tau) - I     (Theorem 3.2)
 * A capped path never reached the boundary (chi_{tau<inf} = 0 in Theorem 3.2
 * as far as the walk could tell): its payoff is -I and capped[t] = 1.
 * tau_steps[t] receives n.  exitpts (nullable) receives X_tau (or the last
 * state when capped).
 */
void orc_observe_dirichlet(const orc_flow *fl, const orc_field *f, const orc_field *g,
                           const double *obs, int n_obs, double kappa, double dt, int64_t Np,
                           uint64_t seed, int64_t max_steps, double *payoff,
                           int64_t *tau_steps, uint8_t *capped, double *exitpts)
{
    int64_t total = (int64_t)n_obs * Np;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < total; ++t) {
        int64_t j = t / Np, i = t % Np;
        double X[2] = {obs[2 * j], obs[2 * j + 1]};
        double I = 0.0;
        int64_t n = 0;
        int exited = 0;
        double E[2] = {X[0], X[1]};
        while (n < max_steps) {
            double Y[2];
            em_step(fl, kappa, dt, seed, (uint64_t)n, (uint32_t)i, (uint32_t)j, X, Y);
            I += orc_field_eval(f, X[0], X[1]) * dt;
            n += 1;
            if (left_domain(fl->domain, Y, E)) {
                exited = 1;
                break;
            }
            X[0] = Y[0]; X[1] = Y[1];
            E[0] = X[0]; E[1] = X[1];
        }
        payoff[t] = (exited ? orc_field_eval(g, E[0], E[1]) : 0.0) - I;
        tau_steps[t] = n;
        capped[t] = (uint8_t)(!exited);
        if (exitpts) {
            exitpts[2 * t] = E[0];
            exitpts[2 * t + 1] = E[1];
        }
    }
}

/* Direct FP64 evaluation at many points (pins and parity of the velocity). */
void orc_velocity_many(const orc_flow *fl, int64_t count, const double *X, double *V)
{
    for (int64_t e = 0; e < count; ++e)
        orc_velocity(fl, X[2 * e], X[2 * e + 1], V + 2 * e);
}

void orc_psi_many(const orc_flow *fl, int64_t count, const double *X, double *P)
{
    for (int64_t e = 0; e < count; ++e)
        P[e] = orc_psi(fl, X[2 * e], X[2 * e + 1]);
}

void orc_field_many(const orc_field *f, int64_t count, const double *X, double *out)
{
    for (int64_t e = 0; e < count; ++e)
        out[e] = orc_field_eval(f, X[2 * e], X[2 * e + 1]);
}

void orc_normals_many(uint64_t seed, int64_t count, const uint64_t *n, const uint32_t *i,
                      const uint32_t *j, double *z)
{
    for (int64_t e = 0; e < count; ++e)
        orc_normals(seed, n[e], i[e], j[e], z + 2 * e);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
