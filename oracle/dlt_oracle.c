/*
 * Direct O(N^2) CPU reference for the discrete Legendre transform.
 * TEST INFRASTRUCTURE ONLY -- see dlt_oracle_impl.h for what is computed
 * and from which passage of the paper.  Built with
 *   gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC
 * (no -ffast-math), so every operation rounds as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REAL double
#define SUFFIX _d
#define PI_R 3.14159265358979323846
#define EPS_R 2.220446049250313e-16
#define SIN_R sin
#define COS_R cos
#define FABS_R fabs
#define IDLT_G 16 /* nodes advanced together by the FP64 inverse (SIMD) */
#include "dlt_oracle_impl.h"
#undef REAL
#undef SUFFIX
#undef PI_R
#undef EPS_R
#undef SIN_R
#undef COS_R
#undef FABS_R
#undef IDLT_G

#define REAL long double
#define SUFFIX _l
#define PI_R 3.14159265358979323846264338327950288L
#define EPS_R 1.0842021724855044340e-19L
#define SIN_R sinl
#define COS_R cosl
#define FABS_R fabsl
#define IDLT_G 1 /* x87: one node at a time */
#include "dlt_oracle_impl.h"

/*
 * Nodes and weights.  Roots of P_N(cos theta) and Gauss-Legendre weights
 * (Sec. 1, eqs. (1)-(2); theta form as argued in Sec. 2.1): Newton's method
 * in theta from the equispaced guess theta^{cheb*}_k = (k+3/4) pi/(N+1/2) of
 * Sec. 2.2, which Lemma 2 places within 1/(3 pi (2N+1)) of the root, using
 * dP_N/dtheta = N (x P_N - P_{N-1}) / sin(theta), until the step is below
 * one ulp.  Weight w_k = 2/(dP_N/dtheta)^2 = 2/((1-x^2) P_N'(x)^2), with the
 * derivative from the same identity evaluated at the final theta (P_N there
 * is kept rather than set to zero, which keeps the weight well conditioned
 * near x = +-1 where P_{N-1} is small).
 * Both builds (_d and _l) use the x87 extended-precision recurrence here:
 * the FP64 recurrence loses about N*eps relative accuracy in P_{N-1}, which
 * the weight would inherit.  Results are rounded to double once at the end.
 */
typedef long double LD;
static const LD PI_LD = 3.14159265358979323846264338327950288L;

static void leg_pair_ld(int64_t N, LD t, LD *pN, LD *pN1) {
    LD s = sinl(t / 2);
    LD u = 2 * s * s;
    LD p = 1, pm = 0, d = 0;
    for (int64_t n = 0; n < N; ++n) {
        d = ((LD)n * d - (LD)(2 * n + 1) * u * p) / (LD)(n + 1);
        pm = p;
        p = p + d;
    }
    *pN = p;
    *pN1 = pm;
}

static void node_half_ld(int64_t N, int64_t k, LD *theta, LD *w) {
    LD t = ((LD)k + 0.75L) * PI_LD / ((LD)N + 0.5L);
    LD pN = 0, pN1 = 0;
    if ((N & 1) && k == (N - 1) / 2) {
        t = PI_LD / 2; /* middle root of an odd-degree P_N is x = 0 */
    } else {
        for (int it = 0; it < 20; ++it) {
            leg_pair_ld(N, t, &pN, &pN1);
            LD dP = (LD)N * (cosl(t) * pN - pN1) / sinl(t);
            LD dt = pN / dP;
            t -= dt;
            if (fabsl(dt) <= 1.0842021724855044340e-19L * t) break;
        }
    }
    leg_pair_ld(N, t, &pN, &pN1);
    LD st = sinl(t);
    LD q = (LD)N * (cosl(t) * pN - pN1);
    *theta = t;
    *w = 2 * st * st / (q * q);
}

static int nodes_impl(int64_t N, int64_t nidx, const int64_t *idx, double *theta, double *w) {
    if (N < 1) return -1;
    int64_t cnt = idx ? nidx : N;
    for (int64_t i = 0; idx && i < cnt; ++i)
        if (idx[i] < 0 || idx[i] >= N) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < cnt; ++i) {
        int64_t k = idx ? idx[i] : i;
        int64_t kk = (k < (N + 1) / 2) ? k : N - 1 - k;
        LD t, ww;
        node_half_ld(N, kk, &t, &ww);
        if (kk != k) t = PI_LD - t;
        if (theta) theta[i] = (double)t;
        if (w) w[i] = (double)ww;
    }
    return 0;
}

int orc_nodes_d(int64_t N, int64_t nidx, const int64_t *idx, double *theta, double *w) {
    return nodes_impl(N, nidx, idx, theta, w);
}

int orc_nodes_l(int64_t N, int64_t nidx, const int64_t *idx, double *theta, double *w) {
    return nodes_impl(N, nidx, idx, theta, w);
}

int orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
