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
 *     velocity Verlet Q = v^T M v + x^T K x - (h^2/4) (K x)^T M^-1 (K x).
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
