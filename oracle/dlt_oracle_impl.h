/*
 * Direct O(N^2) reference for the discrete Legendre transform and its parts.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU path.
 *
 * This file is a template: dlt_oracle.c includes it twice, once with
 * REAL = double (suffix _d, the oracle of record) and once with
 * REAL = long double (suffix _l, the x87 extended-precision cross-check).
 * All interfaces take and return double; REAL is the working precision.
 *
 * What each routine computes, with the passage of Hale & Townsend,
 * "A fast FFT-based discrete Legendre transform" (IMA J. Numer. Anal.), that
 * defines it:
 *   (nodes and weights live in dlt_oracle.c: they are always computed in
 *    extended precision, see there)
 *   dlt       f_k = sum_n c_n P_n(x_k), eq. (1), by the three-term recurrence
 *             ("direct approach", Sec. 2.4 and Sec. 3.1).
 *   idlt      c_n = (n+1/2) sum_k w_k f_k P_n(x_k), eq. (2), recurrence run
 *             along each node and accumulated per degree (Sec. 4.1).
 *   ndct      f_k = sum_n chat_n T_n(x_k) = sum_n chat_n cos(n theta_k),
 *             eq. (3)-(4), Chebyshev three-term recurrence (Sec. 2.4).
 *   leg2cheb  chat = M c with the Legendre-to-Chebyshev matrix of Sec. 3
 *             (Alpert & Rokhlin form).  The entries as printed in the paper
 *             lack one Gamma-ratio factor; the reading used here is
 *             M_kn = (eps_k/pi) Lam((n-k)/2) Lam((n+k)/2), n>=k, n+k even,
 *             Lam(z) = Gamma(z+1/2)/Gamma(z+1), eps_0 = 1, eps_k = 2.
 *             (leg2cheb_rows: the same for a given set of rows;
 *             cheb2leg: c = M^{-1} chat by back substitution.)
 *
 * Recurrences are evaluated for theta' = min(theta, pi - theta) <= pi/2 and
 * mirrored with P_n(-x) = (-1)^n P_n(x), T_n(-x) = (-1)^n T_n(x).  For
 * theta' <= pi/4 they run in u = 2 sin^2(theta/2) = 1 - x (Reinsch's
 * modification): Sec. 2.1 gives the reason for working in theta, since
 * x = cos(theta) loses accuracy near x = +-1.  For pi/4 < theta' <= pi/2 the
 * textbook recurrence in x is used, which rounds less there.
 *
 * Angles are passed as theta (+ optional theta_lo, the low part of a
 * two-double angle theta + theta_lo; NULL means zero), so an evaluation
 * point known to better than double precision can be honoured by the
 * extended build.
 *
 * Parity status of each routine is recorded in the test-suite; every
 * routine here is pinned by at least one test that does not re-run this
 * code's own formula (closed forms, textbook values, library routines,
 * brute force in arbitrary precision, invariants).
 */

#define CAT2(a, b) a##b
#define CAT(a, b) CAT2(a, b)
#define FN(name) CAT(name, SUFFIX)

/* Legendre P_n(cos t) for n = 0..N-1 at one angle, Reinsch form. */
static void FN(leg_row)(int64_t N, REAL t, REAL *P) {
    int flip = t > PI_R / 2;
    REAL tt = flip ? PI_R - t : t;
    if (N > 0) P[0] = 1;
    if (tt <= PI_R / 4) {
        REAL s = SIN_R(tt / 2);
        REAL u = 2 * s * s;
        REAL p = 1, d = 0;
        for (int64_t n = 0; n + 1 < N; ++n) {
            d = ((REAL)n * d - (REAL)(2 * n + 1) * u * p) / (REAL)(n + 1);
            p = p + d;
            P[n + 1] = p;
        }
    } else {
        REAL x = COS_R(tt);
        REAL pm = 0, p = 1;
        for (int64_t n = 0; n + 1 < N; ++n) {
            REAL pn = ((REAL)(2 * n + 1) * x * p - (REAL)n * pm) / (REAL)(n + 1);
            pm = p;
            p = pn;
            P[n + 1] = p;
        }
    }
    if (flip)
        for (int64_t n = 1; n < N; n += 2) P[n] = -P[n];
}

/* f_i = sum_{n<N} c_n P_n(cos theta_i), eq. (1).  For theta' <= pi/4 the
 * recurrence runs in u = 1 - x (Reinsch form); between pi/4 and pi/2 the
 * textbook form in x is used, which rounds less there. */
int FN(orc_dlt)(int64_t N, const double *c, int64_t nt, const double *theta, const double *theta_lo,
                double *f) {
    if (N < 1) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        REAL t = (REAL)theta[i] + (theta_lo ? (REAL)theta_lo[i] : (REAL)0);
        int flip = t > PI_R / 2;
        REAL tt = flip ? PI_R - t : t;
        REAL acc = (REAL)c[0];
        REAL sg = 1;
        if (tt <= PI_R / 4) {
            REAL s = SIN_R(tt / 2);
            REAL u = 2 * s * s;
            REAL p = 1, d = 0;
            for (int64_t n = 0; n + 1 < N; ++n) {
                d = ((REAL)n * d - (REAL)(2 * n + 1) * u * p) / (REAL)(n + 1);
                p = p + d;
                if (flip) sg = -sg;
                acc += (REAL)c[n + 1] * (sg * p);
            }
        } else {
            REAL x = COS_R(tt);
            REAL pm = 0, p = 1;
            for (int64_t n = 0; n + 1 < N; ++n) {
                REAL pn = ((REAL)(2 * n + 1) * x * p - (REAL)n * pm) / (REAL)(n + 1);
                pm = p;
                p = pn;
                if (flip) sg = -sg;
                acc += (REAL)c[n + 1] * (sg * p);
            }
        }
        f[i] = (double)acc;
    }
    return 0;
}

/* f_i = sum_{n<N} chat_n cos(n theta_i), eqs. (3)-(4), by the Chebyshev
 * recurrence T_{n+1} = 2x T_n - T_{n-1}; for theta' <= pi/4 in the form
 * T_{n+1} - T_n = (T_n - T_{n-1}) - 2u T_n with u = 1 - x. */
int FN(orc_ndct)(int64_t N, const double *chat, int64_t nt, const double *theta, const double *theta_lo,
                 double *f) {
    if (N < 1) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        REAL t = (REAL)theta[i] + (theta_lo ? (REAL)theta_lo[i] : (REAL)0);
        int flip = t > PI_R / 2;
        REAL tt = flip ? PI_R - t : t;
        REAL acc = (REAL)chat[0];
        REAL sg = 1;
        if (tt <= PI_R / 4) {
            REAL s = SIN_R(tt / 2);
            REAL u = 2 * s * s;
            REAL p = 1, d = -u;
            for (int64_t n = 1; n < N; ++n) {
                if (n > 1) d = d - 2 * u * p;
                p = p + d;
                if (flip) sg = -sg;
                acc += (REAL)chat[n] * (sg * p);
            }
        } else {
            REAL x = COS_R(tt);
            REAL pm = 1, p = x;
            if (N > 1) {
                if (flip) sg = -sg;
                acc += (REAL)chat[1] * (sg * p);
            }
            for (int64_t n = 2; n < N; ++n) {
                REAL pn = 2 * x * p - pm;
                pm = p;
                p = pn;
                if (flip) sg = -sg;
                acc += (REAL)chat[n] * (sg * p);
            }
        }
        f[i] = (double)acc;
    }
    return 0;
}

/* c_n = (n+1/2) sum_k w_k f_k P_n(cos theta_k), eq. (2), for the requested
 * degrees n (all N if idx == NULL).  One recurrence per node, accumulated
 * per degree ("along rows", Sec. 4.1).
 *
 * The recurrences of IDLT_G neighbouring nodes advance together, one degree
 * at a time, so that their independent chains overlap in the CPU (a loop
 * interchange: every node runs exactly the steps it would run alone); the
 * group's terms of a degree are summed pairwise and then added to that
 * degree's accumulator.  A group whose nodes use both forms of the
 * recurrence runs once per form, the nodes of the other form contributing
 * exact zeros.  IDLT_G (a power of two) is set by the including file. */

/* the angle of node k reduced to [0, pi/2] and its form: 0 = Reinsch (u),
 * 1 = textbook (x); *sgf = -1 when the node lies beyond pi/2 */
static int FN(idlt_form)(const double *theta, const double *theta_lo, int64_t k, REAL *v, REAL *sgf) {
    REAL t = (REAL)theta[k] + (theta_lo ? (REAL)theta_lo[k] : (REAL)0);
    int flip = t > PI_R / 2;
    REAL tt = flip ? PI_R - t : t;
    *sgf = flip ? (REAL)-1 : (REAL)1;
    if (tt <= PI_R / 4) {
        REAL s = SIN_R(tt / 2);
        *v = 2 * s * s;
        return 0;
    }
    *v = COS_R(tt);
    return 1;
}

/* sum of the IDLT_G terms t[0..IDLT_G), pairwise */
static REAL FN(idlt_gsum)(const REAL *t) {
    REAL q[IDLT_G];
    for (int j = 0; j < IDLT_G; ++j) q[j] = t[j];
    for (int h = IDLT_G / 2; h >= 1; h /= 2)
        for (int j = 0; j < h; ++j) q[j] = q[j] + q[j + h];
    return q[0];
}

/* the nodes of one group with weights g[j] (zero: no contribution), all of
 * form `form` with parameters v[j], mirror signs sgf[j]: degrees 0..nmax
 * added to a[] */
static void FN(idlt_group)(int64_t nmax, int form, const REAL *g, const REAL *v, const REAL *sgf, REAL *a) {
    REAL p[IDLT_G], q[IDLT_G], sg[IDLT_G], t[IDLT_G];
    for (int j = 0; j < IDLT_G; ++j) {
        p[j] = 1;
        q[j] = 0; /* d_n (Reinsch form) or P_{n-1} (textbook form) */
        sg[j] = 1;
    }
    a[0] += FN(idlt_gsum)(g);
    if (form == 0) {
        for (int64_t n = 0; n < nmax; ++n) {
#pragma omp simd
            for (int j = 0; j < IDLT_G; ++j) {
                q[j] = ((REAL)n * q[j] - (REAL)(2 * n + 1) * v[j] * p[j]) / (REAL)(n + 1);
                p[j] = p[j] + q[j];
                sg[j] = sg[j] * sgf[j];
                t[j] = g[j] * (sg[j] * p[j]);
            }
            a[n + 1] += FN(idlt_gsum)(t);
        }
    } else {
        for (int64_t n = 0; n < nmax; ++n) {
#pragma omp simd
            for (int j = 0; j < IDLT_G; ++j) {
                REAL pn = ((REAL)(2 * n + 1) * v[j] * p[j] - (REAL)n * q[j]) / (REAL)(n + 1);
                q[j] = p[j];
                p[j] = pn;
                sg[j] = sg[j] * sgf[j];
                t[j] = g[j] * (sg[j] * p[j]);
            }
            a[n + 1] += FN(idlt_gsum)(t);
        }
    }
}

int FN(orc_idlt)(int64_t N, const double *f, const double *theta, const double *theta_lo,
                 const double *w, int64_t nidx, const int64_t *idx, double *c) {
    if (N < 1) return -1;
    int64_t cnt = idx ? nidx : N;
    int64_t nmax = 0;
    for (int64_t i = 0; i < cnt; ++i) {
        int64_t n = idx ? idx[i] : i;
        if (n >= N || n < 0) return -1;
        if (n > nmax) nmax = n;
    }
    /* one accumulator per thread over a static split of the nodes, summed
     * in thread order afterwards, so the result does not depend on timing */
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    REAL *acc = (REAL *)calloc((size_t)nth * (size_t)(nmax + 1), sizeof(REAL));
    if (!acc) return -4;
#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        REAL *a = acc + (size_t)tid * (size_t)(nmax + 1);
        int64_t k0 = N * tid / nth, k1 = N * (tid + 1) / nth;
        for (int64_t kg = k0; kg < k1; kg += IDLT_G) {
            REAL g[IDLT_G], v[IDLT_G], sgf[IDLT_G], gm[IDLT_G], vm[IDLT_G];
            int form[IDLT_G], has[2] = {0, 0};
            for (int j = 0; j < IDLT_G; ++j) {
                g[j] = 0; /* lanes past the thread's last node contribute zero */
                v[j] = 0;
                sgf[j] = 1;
                form[j] = -1;
                if (kg + j < k1) {
                    const int64_t k = kg + j;
                    g[j] = (REAL)w[k] * (REAL)f[k];
                    form[j] = FN(idlt_form)(theta, theta_lo, k, &v[j], &sgf[j]);
                    has[form[j]] = 1;
                }
            }
            for (int fm = 0; fm < 2; ++fm) {
                if (!has[fm]) continue;
                for (int j = 0; j < IDLT_G; ++j) {
                    gm[j] = (form[j] == fm) ? g[j] : 0;
                    vm[j] = (form[j] == fm) ? v[j] : 0;
                }
                FN(idlt_group)(nmax, fm, gm, vm, sgf, a);
            }
        }
    }
    REAL *tot = acc;
    for (int t = 1; t < nth; ++t)
        for (int64_t n = 0; n <= nmax; ++n) tot[n] += acc[(size_t)t * (size_t)(nmax + 1) + (size_t)n];
    for (int64_t i = 0; i < cnt; ++i) {
        int64_t n = idx ? idx[i] : i;
        c[i] = (double)(((REAL)n + (REAL)0.5) * tot[n]);
    }
    free(acc);
    return 0;
}

/* Lam(z) = Gamma(z+1/2)/Gamma(z+1) for z = 0..Z-1 by the ratio
 * Lam(z+1) = Lam(z) (z+1/2)/(z+1), Lam(0) = sqrt(pi); always in long
 * double so the FP64 build keeps M's entries to a few ulps. */
static void FN(lam_table)(int64_t Z, long double *L) {
    long double v = sqrtl(3.14159265358979323846264338327950288L);
    for (int64_t z = 0; z < Z; ++z) {
        L[z] = v;
        v = v * ((long double)z + 0.5L) / ((long double)z + 1.0L);
    }
}

/* chat = M c (dense, O(N^2)), Sec. 3, eq. (9). */
int FN(orc_leg2cheb)(int64_t N, const double *c, double *chat) {
    if (N < 1) return -1;
    long double *L = (long double *)malloc((size_t)N * sizeof(long double));
    if (!L) return -4;
    FN(lam_table)(N, L);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t k = 0; k < N; ++k) {
        REAL acc = 0;
        for (int64_t n = k; n < N; n += 2)
            acc += (REAL)(L[(n - k) / 2] * L[(n + k) / 2]) * (REAL)c[n];
        REAL e = (k == 0) ? 1 : 2;
        chat[k] = (double)(e / PI_R * acc);
    }
    free(L);
    return 0;
}

/* chat_k = (M c)_k for the cnt rows k = idx[i] only, the same definition as
 * orc_leg2cheb (Sec. 3, eq. (9)) restricted to those rows: O(N) per row, so
 * that large N can be checked on a sample of outputs. */
int FN(orc_leg2cheb_rows)(int64_t N, const double *c, int64_t cnt, const int64_t *idx, double *chat) {
    if (N < 1 || cnt < 0 || (cnt > 0 && !idx)) return -1;
    for (int64_t i = 0; i < cnt; ++i)
        if (idx[i] < 0 || idx[i] >= N) return -1;
    long double *L = (long double *)malloc((size_t)N * sizeof(long double));
    if (!L) return -4;
    FN(lam_table)(N, L);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < cnt; ++i) {
        const int64_t k = idx[i];
        REAL acc = 0;
        for (int64_t n = k; n < N; n += 2)
            acc += (REAL)(L[(n - k) / 2] * L[(n + k) / 2]) * (REAL)c[n];
        REAL e = (k == 0) ? 1 : 2;
        chat[i] = (double)(e / PI_R * acc);
    }
    free(L);
    return 0;
}

/* c = M^{-1} chat (Chebyshev to Legendre coefficients): the solution of
 * M c = chat by back substitution, M upper triangular with nonzero diagonal
 * M_kk = (eps_k/pi) Lam(0) Lam(k) (Sec. 3, eq. (9)).  O(N^2). */
int FN(orc_cheb2leg)(int64_t N, const double *chat, double *c) {
    if (N < 1) return -1;
    long double *L = (long double *)malloc((size_t)N * sizeof(long double));
    REAL *x = (REAL *)malloc((size_t)N * sizeof(REAL));
    if (!L || !x) {
        free(L);
        free(x);
        return -4;
    }
    FN(lam_table)(N, L);
    for (int64_t k = N - 1; k >= 0; --k) {
        REAL acc = 0;
        for (int64_t n = k + 2; n < N; n += 2) acc += (REAL)(L[(n - k) / 2] * L[(n + k) / 2]) * x[n];
        REAL e = (k == 0) ? 1 : 2;
        REAL diag = e / PI_R * (REAL)(L[0] * L[k]);
        x[k] = ((REAL)chat[k] - e / PI_R * acc) / diag;
    }
    for (int64_t k = 0; k < N; ++k) c[k] = (double)x[k];
    free(L);
    free(x);
    return 0;
}

/* out = M^T y (dense), used by the inverse transform, Sec. 4. */
int FN(orc_leg2cheb_t)(int64_t N, const double *y, double *out) {
    if (N < 1) return -1;
    long double *L = (long double *)malloc((size_t)N * sizeof(long double));
    if (!L) return -4;
    FN(lam_table)(N, L);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t n = 0; n < N; ++n) {
        REAL acc = 0;
        for (int64_t k = n & 1; k <= n; k += 2) {
            REAL e = (k == 0) ? 1 : 2;
            acc += e * (REAL)(L[(n - k) / 2] * L[(n + k) / 2]) * (REAL)y[k];
        }
        out[n] = (double)(acc / PI_R);
    }
    free(L);
    return 0;
}

/* P_n(cos theta), n = 0..N-1 (exposed for tests). */
int FN(orc_legendre)(int64_t N, double theta, double *P) {
    if (N < 1) return -1;
    REAL *tmp = (REAL *)malloc((size_t)N * sizeof(REAL));
    if (!tmp) return -4;
    FN(leg_row)(N, (REAL)theta, tmp);
    for (int64_t n = 0; n < N; ++n) P[n] = (double)tmp[n];
    free(tmp);
    return 0;
}

#undef FN
