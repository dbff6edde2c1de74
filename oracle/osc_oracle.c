/*
 * FP64 CPU oracle for the coupled harmonic oscillator (arXiv 1702.02207).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the HIP library.
 *
 * What it computes, in the paper's terms:
 *   - eq. (1): sum_j (m_ij x_j'' + k_ij x_j) = 0, i.e. x'' = -A x, A = M^-1 K;
 *   - eq. (2): the fixed-free two-mass chain, generalised to s masses with a
 *     wall spring k[0] on body 0, spring k[i] between bodies i-1 and i, and a
 *     free last body (Fig. 1);
 *   - section 3: reduction to first order, state y = (x, v) with x' = v,
 *     v' = -A x (the RHS D(1..4) written there for eq. (3));
 *   - a fixed-step Runge-Kutta integration of that first-order system.  The
 *     paper does not name the scheme or the step; this oracle uses the classic
 *     four-stage RK4 (nodes 0, 1/2, 1/2, 1; weights 1/6, 1/3, 1/3, 1/6) with a
 *     caller-given step, and velocity Verlet (kick-drift-kick) beside it;
 *   - the energy E = 1/2 v^T M v + 1/2 x^T K x, and the discrete invariant of
 *     velocity Verlet Q = v^T M v + x^T K x - (h^2/4) (K x)^T M^-1 (K x);
 *   - beyond eq. (1): Rayleigh damping and a harmonic force, coupled Van der
 *     Pol chains (the nonlinear oscillators section 1 motivates the work
 *     with), and the adaptive Dormand-Prince pair for MATLAB's solvers (3).
 *
 * Everything is plain double-precision loops, built with -ffp-contract=off so
 * that no fused multiply-add changes the rounding.  OpenMP only spreads
 * independent instances over threads.
 *
 * Frame convention: frames are the states at steps n = 0, stride, 2*stride,
 * ... <= nsteps, stored [frame][instance][dof]; stride 0 means no frames.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOTSPD 2
#define ORC_ENOMEM 4

#define ORC_RK4 0
#define ORC_VERLET 1

/* ----------------------------------------------------------------------- */
/* right-hand sides                                                          */
/* ----------------------------------------------------------------------- */

/* Acceleration of the fixed-free chain (eq. (2) for s bodies):
 *   m_i a_i = -k_i (x_i - x_{i-1}) + k_{i+1} (x_{i+1} - x_i),
 * with x_{-1} = 0 (the wall) and no spring to the right of the last body. */
static void chain_accel(int s, const double *m, const double *k, const double *x, double *a) {
    for (int i = 0; i < s; ++i) {
        double left = (i == 0) ? x[0] : x[i] - x[i - 1];
        double f = -k[i] * left;
        if (i + 1 < s) f += k[i + 1] * (x[i + 1] - x[i]);
        a[i] = f / m[i];
    }
}

/* a = -A x for a dense row-major A. */
static void dense_accel(int s, const double *A, const double *x, double *a) {
    for (int i = 0; i < s; ++i) {
        double acc = 0.0;
        for (int j = 0; j < s; ++j) acc += A[(size_t)i * s + j] * x[j];
        a[i] = -acc;
    }
}

typedef struct {
    int kind;            /* 0 chain, 1 dense */
    int s;
    const double *m, *k; /* chain */
    const double *A;     /* dense */
} rhs_t;

static void accel(const rhs_t *r, const double *x, double *a) {
    if (r->kind == 0) chain_accel(r->s, r->m, r->k, x, a);
    else dense_accel(r->s, r->A, x, a);
}

/* ----------------------------------------------------------------------- */
/* one instance                                                              */
/* ----------------------------------------------------------------------- */

static void store_frame(double *dst, int64_t batch, int64_t b, int s, int64_t f, const double *src) {
    if (!dst) return;
    memcpy(dst + ((size_t)f * batch + b) * s, src, sizeof(double) * s);
}

/* Integrate one instance.  work must hold ORC_WORK_PER_DOF * s doubles. */
#define ORC_WORK_PER_DOF 12
static void integrate_one(const rhs_t *r, int method, double h, const double *x0, const double *v0,
                          int64_t nsteps, int64_t stride, int64_t batch, int64_t b,
                          double *xf, double *vf, double *xe, double *ve, double *work) {
    const int s = r->s;
    double *x = work, *v = work + s;
    /* slopes of the four RK4 stages: k_j = (kjx, kjv) = f(stage argument) */
    double *k1x = work + 2 * s, *k1v = work + 3 * s;
    double *k2x = work + 4 * s, *k2v = work + 5 * s;
    double *k3x = work + 6 * s, *k3v = work + 7 * s;
    double *k4x = work + 8 * s, *k4v = work + 9 * s;
    double *xt = work + 10 * s, *vt = work + 11 * s;   /* stage argument y_n + c h k */
    memcpy(x, x0, sizeof(double) * s);
    memcpy(v, v0, sizeof(double) * s);
    int64_t frame = 0;
    if (stride > 0) {
        store_frame(xf, batch, b, s, frame, x);
        store_frame(vf, batch, b, s, frame, v);
        ++frame;
    }
    if (method == ORC_RK4) {
        for (int64_t n = 1; n <= nsteps; ++n) {
            /* k1 = f(y_n) */
            for (int i = 0; i < s; ++i) k1x[i] = v[i];
            accel(r, x, k1v);
            /* k2 = f(y_n + h/2 k1) */
            for (int i = 0; i < s; ++i) { xt[i] = x[i] + 0.5 * h * k1x[i]; vt[i] = v[i] + 0.5 * h * k1v[i]; }
            for (int i = 0; i < s; ++i) k2x[i] = vt[i];
            accel(r, xt, k2v);
            /* k3 = f(y_n + h/2 k2) */
            for (int i = 0; i < s; ++i) { xt[i] = x[i] + 0.5 * h * k2x[i]; vt[i] = v[i] + 0.5 * h * k2v[i]; }
            for (int i = 0; i < s; ++i) k3x[i] = vt[i];
            accel(r, xt, k3v);
            /* k4 = f(y_n + h k3) */
            for (int i = 0; i < s; ++i) { xt[i] = x[i] + h * k3x[i]; vt[i] = v[i] + h * k3v[i]; }
            for (int i = 0; i < s; ++i) k4x[i] = vt[i];
            accel(r, xt, k4v);
            /* y_{n+1} = y_n + h/6 (k1 + 2 k2 + 2 k3 + k4) */
            for (int i = 0; i < s; ++i) {
                x[i] += h / 6.0 * (k1x[i] + 2.0 * k2x[i] + 2.0 * k3x[i] + k4x[i]);
                v[i] += h / 6.0 * (k1v[i] + 2.0 * k2v[i] + 2.0 * k3v[i] + k4v[i]);
            }
            if (stride > 0 && n % stride == 0) {
                store_frame(xf, batch, b, s, frame, x);
                store_frame(vf, batch, b, s, frame, v);
                ++frame;
            }
        }
    } else {
        double *a = k1v;
        accel(r, x, a);                     /* a_0 = -A x_0 before the first step */
        for (int64_t n = 1; n <= nsteps; ++n) {
            for (int i = 0; i < s; ++i) v[i] += 0.5 * h * a[i];   /* kick  */
            for (int i = 0; i < s; ++i) x[i] += h * v[i];         /* drift */
            accel(r, x, a);
            for (int i = 0; i < s; ++i) v[i] += 0.5 * h * a[i];   /* kick  */
            if (stride > 0 && n % stride == 0) {
                store_frame(xf, batch, b, s, frame, x);
                store_frame(vf, batch, b, s, frame, v);
                ++frame;
            }
        }
    }
    if (xe) memcpy(xe + (size_t)b * s, x, sizeof(double) * s);
    if (ve) memcpy(ve + (size_t)b * s, v, sizeof(double) * s);
}

/* ----------------------------------------------------------------------- */
/* A = M^-1 K by Cholesky (eq. (1) with a full SPD mass matrix)              */
/* ----------------------------------------------------------------------- */

/* M = L L^T (L lower, row-major); returns ORC_ENOTSPD on a non-positive pivot. */
static int cholesky(int s, const double *M, double *L) {
    memset(L, 0, sizeof(double) * (size_t)s * s);
    for (int j = 0; j < s; ++j) {
        double d = M[(size_t)j * s + j];
        for (int p = 0; p < j; ++p) d -= L[(size_t)j * s + p] * L[(size_t)j * s + p];
        if (!(d > 0.0)) return ORC_ENOTSPD;
        double ljj = sqrt(d);
        L[(size_t)j * s + j] = ljj;
        for (int i = j + 1; i < s; ++i) {
            double e = M[(size_t)i * s + j];
            for (int p = 0; p < j; ++p) e -= L[(size_t)i * s + p] * L[(size_t)j * s + p];
            L[(size_t)i * s + j] = e / ljj;
        }
    }
    return ORC_OK;
}

/* A = L^-T (L^-1 K): forward substitution for each column of K, then back
 * substitution with L^T. */
int oracle_form_a(int s, const double *M, const double *K, double *A) {
    if (s < 1 || !M || !K || !A) return ORC_EINVAL;
    double *L = (double *)malloc(sizeof(double) * (size_t)s * s);
    double *Y = (double *)malloc(sizeof(double) * (size_t)s * s);
    if (!L || !Y) { free(L); free(Y); return ORC_ENOMEM; }
    int st = cholesky(s, M, L);
    if (st == ORC_OK) {
        for (int c = 0; c < s; ++c) {
            for (int i = 0; i < s; ++i) {          /* L y = K[:, c] */
                double e = K[(size_t)i * s + c];
                for (int p = 0; p < i; ++p) e -= L[(size_t)i * s + p] * Y[(size_t)p * s + c];
                Y[(size_t)i * s + c] = e / L[(size_t)i * s + i];
            }
            for (int i = s - 1; i >= 0; --i) {     /* L^T a = y */
                double e = Y[(size_t)i * s + c];
                for (int p = i + 1; p < s; ++p) e -= L[(size_t)p * s + i] * A[(size_t)p * s + c];
                A[(size_t)i * s + c] = e / L[(size_t)i * s + i];
            }
        }
    }
    free(L);
    free(Y);
    return st;
}

/* ----------------------------------------------------------------------- */
/* batched drivers                                                           */
/* ----------------------------------------------------------------------- */

static int check_common(int method, int64_t batch, int s, const double *dt, const double *x0,
                        const double *v0, int64_t nsteps, int64_t stride) {
    if (method != ORC_RK4 && method != ORC_VERLET) return ORC_EINVAL;
    if (batch < 0 || s < 1 || nsteps < 0 || stride < 0) return ORC_EINVAL;
    if (batch > 0 && (!dt || !x0 || !v0)) return ORC_EINVAL;
    return ORC_OK;
}

/* Chain instances: m, k [batch][s]; dt [batch]. */
int oracle_chain(int method, int64_t batch, int s, const double *m, const double *k,
                 const double *dt, const double *x0, const double *v0, int64_t nsteps,
                 int64_t stride, double *xf, double *vf, double *xe, double *ve) {
    int st = check_common(method, batch, s, dt, x0, v0, nsteps, stride);
    if (st) return st;
    if (batch > 0 && (!m || !k)) return ORC_EINVAL;
    int fail = 0;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * ORC_WORK_PER_DOF * (size_t)s);
        if (!work) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 0; b < batch; ++b) {
                rhs_t r = {0, s, m + (size_t)b * s, k + (size_t)b * s, NULL};
                integrate_one(&r, method, dt[b], x0 + (size_t)b * s, v0 + (size_t)b * s, nsteps,
                              stride, batch, b, xf, vf, xe, ve, work);
            }
            free(work);
        }
    }
    return fail ? ORC_ENOMEM : ORC_OK;
}

/* Dense instances.  shared != 0: M, K are [s][s] for all instances and dt[0]
 * is the step; otherwise M, K are [batch][s][s] and dt is [batch]. */
int oracle_dense(int method, int64_t batch, int s, int shared, const double *M, const double *K,
                 const double *dt, const double *x0, const double *v0, int64_t nsteps,
                 int64_t stride, double *xf, double *vf, double *xe, double *ve) {
    int st = check_common(method, batch, s, dt, x0, v0, nsteps, stride);
    if (st) return st;
    if (batch > 0 && (!M || !K)) return ORC_EINVAL;
    const size_t ss = (size_t)s * s;
    double *Ashared = NULL;
    if (shared && batch > 0) {
        Ashared = (double *)malloc(sizeof(double) * ss);
        if (!Ashared) return ORC_ENOMEM;
        st = oracle_form_a(s, M, K, Ashared);
        if (st) { free(Ashared); return st; }
    }
    int fail = 0;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * ORC_WORK_PER_DOF * (size_t)s);
        double *Aown = shared ? NULL : (double *)malloc(sizeof(double) * ss);
        if (!work || (!shared && !Aown)) {
#pragma omp atomic write
            fail = ORC_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 0; b < batch; ++b) {
                const double *A = Ashared;
                if (!shared) {
                    int e = oracle_form_a(s, M + b * ss, K + b * ss, Aown);
                    if (e) {
#pragma omp atomic write
                        fail = e;
                        continue;
                    }
                    A = Aown;
                }
                rhs_t r = {1, s, NULL, NULL, A};
                integrate_one(&r, method, shared ? dt[0] : dt[b], x0 + (size_t)b * s,
                              v0 + (size_t)b * s, nsteps, stride, batch, b, xf, vf, xe, ve, work);
            }
        }
        free(work);
        free(Aown);
    }
    free(Ashared);
    return fail;
}

/* ----------------------------------------------------------------------- */
/* energy and the Verlet invariant                                           */
/* ----------------------------------------------------------------------- */

/* Chain: E = 1/2 sum m_i v_i^2 + 1/2 sum k_i (x_i - x_{i-1})^2, x_{-1} = 0. */
int oracle_energy_chain(int64_t batch, int s, const double *m, const double *k, const double *x,
                        const double *v, double *E) {
    if (batch < 0 || s < 1) return ORC_EINVAL;
    for (int64_t b = 0; b < batch; ++b) {
        const double *mb = m + b * s, *kb = k + b * s, *xb = x + b * s, *vb = v + b * s;
        double kin = 0.0, pot = 0.0;
        for (int i = 0; i < s; ++i) {
            double ext = (i == 0) ? xb[0] : xb[i] - xb[i - 1];
            kin += mb[i] * vb[i] * vb[i];
            pot += kb[i] * ext * ext;
        }
        E[b] = 0.5 * kin + 0.5 * pot;
    }
    return ORC_OK;
}

/* Dense: E = 1/2 v^T M v + 1/2 x^T K x; M, K shared [s][s] or per instance. */
int oracle_energy_dense(int64_t batch, int s, int shared, const double *M, const double *K,
                        const double *x, const double *v, double *E) {
    if (batch < 0 || s < 1) return ORC_EINVAL;
    const size_t ss = (size_t)s * s;
    for (int64_t b = 0; b < batch; ++b) {
        const double *Mb = shared ? M : M + b * ss, *Kb = shared ? K : K + b * ss;
        const double *xb = x + b * s, *vb = v + b * s;
        double kin = 0.0, pot = 0.0;
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < s; ++j) {
                kin += vb[i] * Mb[(size_t)i * s + j] * vb[j];
                pot += xb[i] * Kb[(size_t)i * s + j] * xb[j];
            }
        E[b] = 0.5 * kin + 0.5 * pot;
    }
    return ORC_OK;
}

/* Verlet invariant for a chain: Q = v^T M v + x^T K x - (h^2/4) f^T M^-1 f with
 * f = K x (the spring forces on each body, with sign). */
int oracle_verlet_q_chain(int64_t batch, int s, const double *m, const double *k, const double *dt,
                          const double *x, const double *v, double *Q) {
    if (batch < 0 || s < 1) return ORC_EINVAL;
    double *a = (double *)malloc(sizeof(double) * s);
    if (!a) return ORC_ENOMEM;
    for (int64_t b = 0; b < batch; ++b) {
        const double *mb = m + b * s, *kb = k + b * s, *xb = x + b * s, *vb = v + b * s;
        chain_accel(s, mb, kb, xb, a);         /* a = -M^-1 K x */
        double kin = 0.0, pot = 0.0, corr = 0.0;
        for (int i = 0; i < s; ++i) {
            double ext = (i == 0) ? xb[0] : xb[i] - xb[i - 1];
            kin += mb[i] * vb[i] * vb[i];
            pot += kb[i] * ext * ext;
            corr += mb[i] * a[i] * a[i];       /* (Kx)^T M^-1 (Kx) = a^T M a */
        }
        Q[b] = kin + pot - 0.25 * dt[b] * dt[b] * corr;
    }
    free(a);
    return ORC_OK;
}

/* Verlet invariant for dense systems (eq. (1) with full M, K): with f = K x
 * and A = M^-1 K formed by Cholesky as above, (K x)^T M^-1 (K x) = f^T (A x),
 * so Q = v^T M v + x^T K x - (h^2/4) f^T (A x).  M, K shared [s][s] (dt[0])
 * or per instance [batch][s][s] (dt[b]). */
int oracle_verlet_q_dense(int64_t batch, int s, int shared, const double *M, const double *K,
                          const double *dt, const double *x, const double *v, double *Q) {
    if (batch < 0 || s < 1) return ORC_EINVAL;
    const size_t ss = (size_t)s * s;
    double *A = (double *)malloc(sizeof(double) * ss);
    double *f = (double *)malloc(sizeof(double) * s);
    double *ax = (double *)malloc(sizeof(double) * s);
    if (!A || !f || !ax) { free(A); free(f); free(ax); return ORC_ENOMEM; }
    int st = ORC_OK;
    for (int64_t b = 0; b < batch && st == ORC_OK; ++b) {
        const double *Mb = shared ? M : M + b * ss, *Kb = shared ? K : K + b * ss;
        if (b == 0 || !shared) st = oracle_form_a(s, Mb, Kb, A);
        if (st) break;
        const double *xb = x + b * s, *vb = v + b * s;
        const double h = shared ? dt[0] : dt[b];
        double kin = 0.0, pot = 0.0, corr = 0.0;
        for (int i = 0; i < s; ++i) {
            double fi = 0.0, ai = 0.0;
            for (int j = 0; j < s; ++j) {
                fi += Kb[(size_t)i * s + j] * xb[j];
                ai += A[(size_t)i * s + j] * xb[j];
            }
            f[i] = fi;
            ax[i] = ai;
        }
        for (int i = 0; i < s; ++i) {
            for (int j = 0; j < s; ++j) {
                kin += vb[i] * Mb[(size_t)i * s + j] * vb[j];
                pot += xb[i] * Kb[(size_t)i * s + j] * xb[j];
            }
            corr += f[i] * ax[i];
        }
        Q[b] = kin + pot - 0.25 * h * h * corr;
    }
    free(A);
    free(f);
    free(ax);
    return st;
}

/* ----------------------------------------------------------------------- */
/* the scheme as a matrix                                                    */
/* ----------------------------------------------------------------------- */

/* For eq. (1) the first-order system of section 3 is y' = L y with the
 * constant matrix L = [[0, I], [-A, 0]], y = (x, v), and both schemes map y
 * linearly: k steps are one matrix P_k, y_{n+k} = P_k y_n.  Column j of P_k
 * is the state after k steps started from the j-th unit vector of R^2s; that
 * is how it is formed here, with the integrator above.
 * kind 0: chain (a = m, b = k, each [s]); kind 1: dense (a = M, b = K, each
 * [s][s], A = M^-1 K by Cholesky).  P: [2s][2s] row-major, positions first. */
int oracle_propagator(int method, int kind, int s, const double *a, const double *b, double dt,
                      int64_t k, double *P) {
    if ((method != ORC_RK4 && method != ORC_VERLET) || (kind != 0 && kind != 1) || s < 1 || k < 0 ||
        !a || !b || !P || !(dt > 0.0))
        return ORC_EINVAL;
    const int n = 2 * s;
    double *A = NULL;
    if (kind == 1) {
        A = (double *)malloc(sizeof(double) * (size_t)s * s);
        if (!A) return ORC_ENOMEM;
        int st = oracle_form_a(s, a, b, A);
        if (st) { free(A); return st; }
    }
    rhs_t r = {kind, s, kind == 0 ? a : NULL, kind == 0 ? b : NULL, A};
    int fail = 0;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * ORC_WORK_PER_DOF * (size_t)s);
        double *y0 = (double *)malloc(sizeof(double) * n);
        double *ye = (double *)malloc(sizeof(double) * n);
        if (!work || !y0 || !ye) {
#pragma omp atomic write
            fail = ORC_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int j = 0; j < n; ++j) {
                for (int i = 0; i < n; ++i) y0[i] = (i == j) ? 1.0 : 0.0;
                integrate_one(&r, method, dt, y0, y0 + s, k, 0, 1, 0, NULL, NULL, ye, ye + s, work);
                for (int i = 0; i < n; ++i) P[(size_t)i * n + j] = ye[i];
            }
        }
        free(work);
        free(y0);
        free(ye);
    }
    free(A);
    return fail;
}

/* ----------------------------------------------------------------------- */
/* damped and driven systems                                                 */
/* ----------------------------------------------------------------------- */

/* Beyond the paper's free vibrations (eq. (1)): Rayleigh damping C = alpha M
 * + beta K and a harmonic force F cos(Omega t),
 *     M x'' + C x' + K x = F cos(Omega t),
 * i.e. in the first-order form of section 3
 *     x' = v,   v' = -A x - (alpha v + beta A v) + f cos(Omega t),  f = M^-1 F.
 * With alpha = beta = 0 and no force the acceleration is computed by the same
 * operations as above, so the results equal those of the free integrator. */
typedef struct {
    double alpha, beta, omega;
    const double *f;     /* [s] or NULL */
    double mu;           /* chains: Van der Pol coefficient (0: none) */
} drive_t;

static void accel_driven(const rhs_t *r, const drive_t *d, double t, const double *x, const double *v,
                         double *a, double *tmp) {
    accel(r, x, a);                                  /* -A x */
    if (d->alpha != 0.0 || d->beta != 0.0) {
        accel(r, v, tmp);                            /* -A v */
        for (int i = 0; i < r->s; ++i) a[i] += -d->alpha * v[i] + d->beta * tmp[i];
    }
    if (d->f) {
        const double c = cos(d->omega * t);
        for (int i = 0; i < r->s; ++i) a[i] += d->f[i] * c;
    }
    if (d->mu != 0.0 && r->kind == 0) {
        /* Van der Pol element on every body of a chain: the force
         * mu (1 - x_i^2) x_i' pumps energy in while |x_i| < 1 and takes it
         * out beyond, which draws each body towards a limit cycle */
        for (int i = 0; i < r->s; ++i) a[i] += d->mu * ((1.0 - x[i] * x[i]) * v[i]) / r->m[i];
    }
}

/* Classic RK4 on the driven first-order system; the stages are evaluated at
 * t_n, t_n + h/2, t_n + h/2 and t_n + h with t_n = n h. */
#define ORC_DRIVEN_WORK_PER_DOF 13
static void integrate_driven_one(const rhs_t *r, const drive_t *d, double h, const double *x0,
                                 const double *v0, int64_t nsteps, int64_t stride, int64_t batch,
                                 int64_t b, double *xf, double *vf, double *xe, double *ve, double *work) {
    const int s = r->s;
    double *x = work, *v = work + s;
    double *k1x = work + 2 * s, *k1v = work + 3 * s, *k2x = work + 4 * s, *k2v = work + 5 * s;
    double *k3x = work + 6 * s, *k3v = work + 7 * s, *k4x = work + 8 * s, *k4v = work + 9 * s;
    double *xt = work + 10 * s, *vt = work + 11 * s, *tmp = work + 12 * s;
    memcpy(x, x0, sizeof(double) * s);
    memcpy(v, v0, sizeof(double) * s);
    int64_t frame = 0;
    if (stride > 0) {
        store_frame(xf, batch, b, s, frame, x);
        store_frame(vf, batch, b, s, frame, v);
        ++frame;
    }
    for (int64_t n = 0; n < nsteps; ++n) {
        const double t = (double)n * h;
        for (int i = 0; i < s; ++i) k1x[i] = v[i];
        accel_driven(r, d, t, x, v, k1v, tmp);
        for (int i = 0; i < s; ++i) { xt[i] = x[i] + 0.5 * h * k1x[i]; vt[i] = v[i] + 0.5 * h * k1v[i]; }
        for (int i = 0; i < s; ++i) k2x[i] = vt[i];
        accel_driven(r, d, t + 0.5 * h, xt, vt, k2v, tmp);
        for (int i = 0; i < s; ++i) { xt[i] = x[i] + 0.5 * h * k2x[i]; vt[i] = v[i] + 0.5 * h * k2v[i]; }
        for (int i = 0; i < s; ++i) k3x[i] = vt[i];
        accel_driven(r, d, t + 0.5 * h, xt, vt, k3v, tmp);
        for (int i = 0; i < s; ++i) { xt[i] = x[i] + h * k3x[i]; vt[i] = v[i] + h * k3v[i]; }
        for (int i = 0; i < s; ++i) k4x[i] = vt[i];
        accel_driven(r, d, t + h, xt, vt, k4v, tmp);
        for (int i = 0; i < s; ++i) {
            x[i] += h / 6.0 * (k1x[i] + 2.0 * k2x[i] + 2.0 * k3x[i] + k4x[i]);
            v[i] += h / 6.0 * (k1v[i] + 2.0 * k2v[i] + 2.0 * k3v[i] + k4v[i]);
        }
        if (stride > 0 && (n + 1) % stride == 0) {
            store_frame(xf, batch, b, s, frame, x);
            store_frame(vf, batch, b, s, frame, v);
            ++frame;
        }
    }
    if (xe) memcpy(xe + (size_t)b * s, x, sizeof(double) * s);
    if (ve) memcpy(ve + (size_t)b * s, v, sizeof(double) * s);
}

/* f = M^-1 F for a dense SPD M (Cholesky, forward and back substitution). */
static int solve_spd(int s, const double *M, const double *F, double *f, double *L, double *y) {
    int st = cholesky(s, M, L);
    if (st) return st;
    for (int i = 0; i < s; ++i) {
        double e = F[i];
        for (int p = 0; p < i; ++p) e -= L[(size_t)i * s + p] * y[p];
        y[i] = e / L[(size_t)i * s + i];
    }
    for (int i = s - 1; i >= 0; --i) {
        double e = y[i];
        for (int p = i + 1; p < s; ++p) e -= L[(size_t)p * s + i] * f[p];
        f[i] = e / L[(size_t)i * s + i];
    }
    return ORC_OK;
}

/* Driven chains: m, k, F [batch][s] (F may be NULL), dt, omega [batch]. */
int oracle_chain_driven(int64_t batch, int s, const double *m, const double *k, const double *dt,
                        double alpha, double beta, const double *F, const double *omega,
                        const double *x0, const double *v0, int64_t nsteps, int64_t stride,
                        double *xf, double *vf, double *xe, double *ve) {
    int st = check_common(ORC_RK4, batch, s, dt, x0, v0, nsteps, stride);
    if (st) return st;
    if (batch > 0 && (!m || !k || (F && !omega))) return ORC_EINVAL;
    int fail = 0;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * ORC_DRIVEN_WORK_PER_DOF * (size_t)s);
        double *f = (double *)malloc(sizeof(double) * s);
        if (!work || !f) {
#pragma omp atomic write
            fail = ORC_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 0; b < batch; ++b) {
                const double *mb = m + (size_t)b * s;
                if (F)
                    for (int i = 0; i < s; ++i) f[i] = F[(size_t)b * s + i] / mb[i];
                drive_t d = {alpha, beta, F ? omega[b] : 0.0, F ? f : NULL, 0.0};
                rhs_t r = {0, s, mb, k + (size_t)b * s, NULL};
                integrate_driven_one(&r, &d, dt[b], x0 + (size_t)b * s, v0 + (size_t)b * s, nsteps, stride,
                                     batch, b, xf, vf, xe, ve, work);
            }
        }
        free(work);
        free(f);
    }
    return fail;
}

/* Coupled Van der Pol chains (the nonlinear oscillators section 1 names as the
 * standard model of the field): the chain of eq. (2) with a Van der Pol
 * element on every body, optionally driven by a harmonic force,
 *     m_i x_i'' - mu (1 - x_i^2) x_i' + (K x)_i = F_i cos(Omega t),
 * by classic RK4 on the first-order system (stages as above; F [batch][s] or
 * NULL, omega [batch]).  mu = 0 gives the free (or driven) chain by the same
 * operations as the damped, driven integrator. */
int oracle_chain_vdp(int64_t batch, int s, const double *m, const double *k, const double *dt, double mu,
                     const double *F, const double *omega, const double *x0, const double *v0, int64_t nsteps,
                     int64_t stride, double *xf, double *vf, double *xe, double *ve) {
    int st = check_common(ORC_RK4, batch, s, dt, x0, v0, nsteps, stride);
    if (st) return st;
    if (batch > 0 && (!m || !k || (F && !omega))) return ORC_EINVAL;
    if (!(mu >= 0.0) || !isfinite(mu)) return ORC_EINVAL;
    int fail = 0;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * ORC_DRIVEN_WORK_PER_DOF * (size_t)s);
        double *f = (double *)malloc(sizeof(double) * s);
        if (!work || !f) {
#pragma omp atomic write
            fail = ORC_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 0; b < batch; ++b) {
                const double *mb = m + (size_t)b * s;
                if (F)
                    for (int i = 0; i < s; ++i) f[i] = F[(size_t)b * s + i] / mb[i];
                drive_t d = {0.0, 0.0, F ? omega[b] : 0.0, F ? f : NULL, mu};
                rhs_t r = {0, s, mb, k + (size_t)b * s, NULL};
                integrate_driven_one(&r, &d, dt[b], x0 + (size_t)b * s, v0 + (size_t)b * s, nsteps, stride,
                                     batch, b, xf, vf, xe, ve, work);
            }
        }
        free(work);
        free(f);
    }
    return fail;
}

/* Driven dense systems: M, K shared [s][s] (dt[0]) or per instance; F [batch][s]
 * (may be NULL), omega [batch]. */
int oracle_dense_driven(int64_t batch, int s, int shared, const double *M, const double *K,
                        const double *dt, double alpha, double beta, const double *F,
                        const double *omega, const double *x0, const double *v0, int64_t nsteps,
                        int64_t stride, double *xf, double *vf, double *xe, double *ve) {
    int st = check_common(ORC_RK4, batch, s, dt, x0, v0, nsteps, stride);
    if (st) return st;
    if (batch > 0 && (!M || !K || (F && !omega))) return ORC_EINVAL;
    const size_t ss = (size_t)s * s;
    int fail = 0;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * ORC_DRIVEN_WORK_PER_DOF * (size_t)s);
        double *A = (double *)malloc(sizeof(double) * ss);
        double *L = (double *)malloc(sizeof(double) * ss);
        double *f = (double *)malloc(sizeof(double) * s);
        double *y = (double *)malloc(sizeof(double) * s);
        if (!work || !A || !L || !f || !y) {
#pragma omp atomic write
            fail = ORC_ENOMEM;
        } else {
            int64_t formed = -1;
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 0; b < batch; ++b) {
                const int64_t sys = shared ? 0 : b;
                const double *Mb = M + sys * ss, *Kb = K + sys * ss;
                int e = ORC_OK;
                if (formed != sys) {
                    e = oracle_form_a(s, Mb, Kb, A);
                    formed = sys;
                }
                if (!e && F) e = solve_spd(s, Mb, F + (size_t)b * s, f, L, y);
                if (e) {
#pragma omp atomic write
                    fail = e;
                    formed = -1;
                    continue;
                }
                drive_t d = {alpha, beta, F ? omega[b] : 0.0, F ? f : NULL, 0.0};
                rhs_t r = {1, s, NULL, NULL, A};
                integrate_driven_one(&r, &d, shared ? dt[0] : dt[b], x0 + (size_t)b * s, v0 + (size_t)b * s,
                                     nsteps, stride, batch, b, xf, vf, xe, ve, work);
            }
        }
        free(work);
        free(A);
        free(L);
        free(f);
        free(y);
    }
    return fail;
}

/* ----------------------------------------------------------------------- */
/* adaptive reference: Dormand-Prince 5(4)                                   */
/* ----------------------------------------------------------------------- */

/* The explicit embedded Runge-Kutta pair of Dormand and Prince (1980), the
 * method behind MATLAB's ode45, with which section 3 integrates its model:
 * seven stages (the last one reused as the first of the next step), the
 * fifth-order solution propagated, the difference to the fourth-order one as
 * the error estimate.  Error norm: root mean square over the 2s components of
 * err_i / (atol + rtol max(|y_i|, |y_new_i|)); a step is accepted when the
 * norm is <= 1, and the next step is h * min(5, max(0.2, 0.9 norm^-1/5)).
 * Output at t_j = j t_end / nout (j = 0..nout): steps are shortened to land on
 * each output time.  One instance of a chain (kind 0: a = m, b = k) or a dense
 * system (kind 1: a = M, b = K), damped and driven as above (F may be NULL).
 * xo, vo: [nout+1][s].  stats: accepted and rejected steps. */
/* The integration itself, for one instance with right-hand side r and drive d. */
static int dopri_core(const rhs_t *r, const drive_t *d, const double *x0, const double *v0, double t_end,
                      int nout, double rtol, double atol, double *xo, double *vo, int64_t *stats) {
    static const double c2 = 1.0 / 5, c3 = 3.0 / 10, c4 = 4.0 / 5, c5 = 8.0 / 9;
    static const double a21 = 1.0 / 5;
    static const double a31 = 3.0 / 40, a32 = 9.0 / 40;
    static const double a41 = 44.0 / 45, a42 = -56.0 / 15, a43 = 32.0 / 9;
    static const double a51 = 19372.0 / 6561, a52 = -25360.0 / 2187, a53 = 64448.0 / 6561, a54 = -212.0 / 729;
    static const double a61 = 9017.0 / 3168, a62 = -355.0 / 33, a63 = 46732.0 / 5247, a64 = 49.0 / 176,
                        a65 = -5103.0 / 18656;
    static const double a71 = 35.0 / 384, a73 = 500.0 / 1113, a74 = 125.0 / 192, a75 = -2187.0 / 6784,
                        a76 = 11.0 / 84;
    static const double e1 = 71.0 / 57600, e3 = -71.0 / 16695, e4 = 71.0 / 1920, e5 = -17253.0 / 339200,
                        e6 = 22.0 / 525, e7 = -1.0 / 40;
    const int s = r->s, n = 2 * s;
    double *buf = (double *)calloc((size_t)n * 10 + (size_t)s, sizeof(double));
    if (!buf) return ORC_ENOMEM;
    double *y = buf, *yn = y + n, *yt = yn + n, *k[7];
    for (int q = 0; q < 7; ++q) k[q] = yt + n + (size_t)q * n;
    double *tmp = k[6] + n;
    int st = ORC_OK;
    /* derivative of the first-order state z = (x, v) */
#define DERIV(t_, z_, out_)                                                   \
    do {                                                                      \
        memcpy((out_), (z_) + s, sizeof(double) * s);                         \
        accel_driven(r, d, (t_), (z_), (z_) + s, (out_) + s, tmp);          \
    } while (0)
    memcpy(y, x0, sizeof(double) * s);
    memcpy(y + s, v0, sizeof(double) * s);
    memcpy(xo, x0, sizeof(double) * s);
    memcpy(vo, v0, sizeof(double) * s);
    double t = 0.0;
    DERIV(t, y, k[0]);
    double h = 0.01 * t_end / nout;   /* first trial step; the controller adapts it */
    int64_t acc = 0, rej = 0;
    for (int j = 1; j <= nout && !st; ++j) {
        const double tj = t_end * (double)j / (double)nout;
        while (t < tj) {
            int last = 0;
            double hs = h;
            if (t + hs >= tj) { hs = tj - t; last = 1; }
            for (int i = 0; i < n; ++i) yt[i] = y[i] + hs * a21 * k[0][i];
            DERIV(t + c2 * hs, yt, k[1]);
            for (int i = 0; i < n; ++i) yt[i] = y[i] + hs * (a31 * k[0][i] + a32 * k[1][i]);
            DERIV(t + c3 * hs, yt, k[2]);
            for (int i = 0; i < n; ++i) yt[i] = y[i] + hs * (a41 * k[0][i] + a42 * k[1][i] + a43 * k[2][i]);
            DERIV(t + c4 * hs, yt, k[3]);
            for (int i = 0; i < n; ++i)
                yt[i] = y[i] + hs * (a51 * k[0][i] + a52 * k[1][i] + a53 * k[2][i] + a54 * k[3][i]);
            DERIV(t + c5 * hs, yt, k[4]);
            for (int i = 0; i < n; ++i)
                yt[i] = y[i] + hs * (a61 * k[0][i] + a62 * k[1][i] + a63 * k[2][i] + a64 * k[3][i] + a65 * k[4][i]);
            DERIV(t + hs, yt, k[5]);
            for (int i = 0; i < n; ++i)
                yn[i] = y[i] + hs * (a71 * k[0][i] + a73 * k[2][i] + a74 * k[3][i] + a75 * k[4][i] + a76 * k[5][i]);
            DERIV(t + hs, yn, k[6]);
            double norm = 0.0;
            for (int i = 0; i < n; ++i) {
                const double err = hs * (e1 * k[0][i] + e3 * k[2][i] + e4 * k[3][i] + e5 * k[4][i] +
                                         e6 * k[5][i] + e7 * k[6][i]);
                const double sc = atol + rtol * fmax(fabs(y[i]), fabs(yn[i]));
                norm += (err / sc) * (err / sc);
            }
            norm = sqrt(norm / n);
            const double fac = norm > 0.0 ? fmin(5.0, fmax(0.2, 0.9 * pow(norm, -0.2))) : 5.0;
            if (norm <= 1.0) {
                t = last ? tj : t + hs;
                memcpy(y, yn, sizeof(double) * n);
                memcpy(k[0], k[6], sizeof(double) * n);   /* first stage of the next step */
                ++acc;
                if (!last || fac < 1.0) h = hs * fac;
            } else {
                h = hs * fac;
                ++rej;
            }
            if (!(h > 1e-14 * t_end) || acc + rej > 100000000) { st = ORC_EINVAL; break; }
        }
        memcpy(xo + (size_t)j * s, y, sizeof(double) * s);
        memcpy(vo + (size_t)j * s, y + s, sizeof(double) * s);
    }
#undef DERIV
    if (stats) { stats[0] = acc; stats[1] = rej; }
    free(buf);
    return st;
}

int oracle_dopri_driven(int kind, int s, const double *a, const double *b, double alpha, double beta,
                        const double *F, double omega, const double *x0, const double *v0, double t_end,
                        int nout, double rtol, double atol, double *xo, double *vo, int64_t *stats) {
    if ((kind != 0 && kind != 1) || s < 1 || nout < 1 || !(t_end > 0.0) || !(rtol > 0.0) || !(atol >= 0.0) ||
        !a || !b || !x0 || !v0 || !xo || !vo)
        return ORC_EINVAL;
    const size_t ss = (size_t)s * s;
    double *buf = (double *)calloc(ss * 2 + 2 * (size_t)s, sizeof(double));
    if (!buf) return ORC_ENOMEM;
    double *A = buf, *L = A + ss, *f = L + ss, *yy = f + s;
    rhs_t r;
    int st = ORC_OK;
    if (kind == 1) {
        st = oracle_form_a(s, a, b, A);
        if (!st && F) st = solve_spd(s, a, F, f, L, yy);
        r = (rhs_t){1, s, NULL, NULL, A};
    } else {
        if (F)
            for (int i = 0; i < s; ++i) f[i] = F[i] / a[i];
        r = (rhs_t){0, s, a, b, NULL};
    }
    if (!st) {
        drive_t d = {alpha, beta, omega, F ? f : NULL, 0.0};
        st = dopri_core(&r, &d, x0, v0, t_end, nout, rtol, atol, xo, vo, stats);
    }
    free(buf);
    return st;
}

/* The same adaptive reference for one Van der Pol chain (m, k [s], mu). */
int oracle_dopri_vdp(int s, const double *m, const double *k, double mu, const double *x0, const double *v0,
                     double t_end, int nout, double rtol, double atol, double *xo, double *vo, int64_t *stats) {
    if (s < 1 || nout < 1 || !(t_end > 0.0) || !(rtol > 0.0) || !(atol >= 0.0) || !(mu >= 0.0) ||
        !isfinite(mu) || !m || !k || !x0 || !v0 || !xo || !vo)
        return ORC_EINVAL;
    rhs_t r = {0, s, m, k, NULL};
    drive_t d = {0.0, 0.0, 0.0, NULL, mu};
    return dopri_core(&r, &d, x0, v0, t_end, nout, rtol, atol, xo, vo, stats);
}
