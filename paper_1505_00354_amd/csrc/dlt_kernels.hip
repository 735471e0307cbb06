// Kernels of the fast discrete Legendre transform (Hale & Townsend):
//   nodes      Legendre nodes/weights and dtheta = theta^leg - theta^cheb1
//   dense      exact Legendre-to-Chebyshev conversion of the low columns
//   far A/B    asymptotic (Stieltjes) blocks of the conversion, one length-N
//              DFT per (block, term), two passes through HBM
//   near       direct three-term recurrence where the expansion is invalid
//   dct2 A/B   values on the Chebyshev grid -> Chebyshev coefficients
//   ndct A/B   Taylor-series evaluation at the Legendre nodes (Sec. 2),
//              two Taylor terms per complex DFT, Horner combine per node
// Grid notation: theta_j = (j+1/2) pi / N, j in [0, N).  A length-N complex
// DFT with + sign, output index m, covers row j(m) = 2m (m < N/2) or
// 2N-1-2m (m >= N/2); this is how sums over e^{i n theta_j} are formed.
#include "dlt_kernels.hpp"

#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace dlt {

__device__ __forceinline__ int row_of(int m, int N) { return (2 * m < N) ? 2 * m : 2 * N - 1 - 2 * m; }

// e^{i pi n/(2N)}
__device__ __forceinline__ cplx half_shift(int64_t n, int N) {
    double s, c;
    sincospi((double)n / (2.0 * N), &s, &c);
    return {c, s};
}

// e^{i pi n/(2N)}, 0 <= n < 4N, from the plan's tables:
// e^{2 pi i floor(n/4)/N} e^{i pi (n mod 4)/(2N)}
__device__ __forceinline__ cplx half_shift_tab(const Geo& g, int n) {
    return cmul(tw2(g.twHi, g.twLo, n >> 2, g.sh), g.qs[n & 3]);
}
// e^{i pi s/16}, s = 0..7: in a tile of compile-time length L the thread's
// elements are n0 + s N/8 (pass A: n = n_a + N1 (i0 + s L/8) with L = N2,
// N1 L = N; pass B: n = j_b + N2 (i0 + s L/8) with L = N1), so
// e^{i pi n/(2N)} = e^{i pi n0/(2N)} e^{i pi s/16}
__device__ constexpr cplx HALF_SHIFT_STEP[8] = {
    {1.0, 0.0},
    {0.9807852804032304, 0.19509032201612825},
    {0.9238795325112867, 0.3826834323650898},
    {0.8314696123025452, 0.5555702330196022},
    {0.7071067811865476, 0.7071067811865475},
    {0.5555702330196023, 0.8314696123025452},
    {0.38268343236508984, 0.9238795325112867},
    {0.19509032201612833, 0.9807852804032304}
};
// e^{i pi n/(2N)} of the elements n0 + s N/8, s = 0..7 (a thread's elements
// in a tile of compile-time length, in either pass): one table value times
// the constants above
__device__ __forceinline__ void half_shift_eighths(const Geo& g, int n0, cplx* e) {
    const cplx e0 = half_shift_tab(g, n0);
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) e[s] = (s == 0) ? e0 : cmul(e0, HALF_SHIFT_STEP[s]);
}

// ------------------------------------------------------------------ nodes --
// Interior nodes k in [kb, ceil(N/2)): Newton in delta = theta - theta*_k
// (theta*_k = (k+1/2)pi/N) on the M-term Stieltjes expansion of P_N(cos theta)
// with the large phase (N+m+1/2) theta reduced exactly:
//   (N+m+1/2) theta*_k - (m+1/2) pi/2 = (k+1/2) pi + (m+1/2)(theta*_k - pi/2),
// so cos(phase) = -(-1)^k sin psi_m, sin(phase) = (-1)^k cos psi_m with
// psi_m = (m+1/2)(theta - pi/2) + N delta.
// P_N(cos theta) / (-(-1)^k C) and its theta-derivative / (-(-1)^k C) at
// theta = theta*_k + delta from the Stieltjes series (terms below rounding
// dropped).
__device__ __forceinline__ void node_series(const NodeParams& P, double a0, double ts, double delta, double& Pv,
                                            double& Dv) {
    const int N = P.N;
    double th = ts + delta;
    double sn, cs;
    sincos(th, &sn, &cs);
    double cot = cs / sn;
    double q = 1.0 / (2.0 * sn);
    double dlt = a0 + delta;  // theta - pi/2
    double ps, pc, rs, rc;
    sincos(0.5 * dlt + N * delta, &ps, &pc);
    sincos(dlt, &rs, &rc);
    double r = sqrt(q);
    const double stop = 1e-18 * P.h[0] * r;
    Pv = 0;
    Dv = 0;
    for (int m = 0; m < P.Ms; ++m) {
        double hm = P.h[m] * r;
        Pv = fma(hm, ps, Pv);
        Dv = fma(hm, (N + m + 0.5) * pc - (m + 0.5) * ps * cot, Dv);
        if (hm < stop) break;  // remaining terms below rounding
        double nps = ps * rc + pc * rs;
        double npc = pc * rc - ps * rs;
        ps = nps;
        pc = npc;
        r *= q;
    }
}

// theta_k - theta*_k (delta) and w_k of interior node k of P_N.  The start
// is within half an ulp of theta_k for all but about the 2000 nodes nearest
// each end, and two Newton steps converge everywhere (k >= 6); a wave whose
// first steps are all below half an ulp (over its active lanes) is done after
// one evaluation, whose derivative then gives the weight.
__device__ void node_interior(const NodeParams& P, int k, double& delta_out, double& w_out) {
    const int N = P.N;
    const double pi = 3.141592653589793;
    const double nu = N + 0.5;
    // start: psi + cot(psi)/(8 nu^2), psi = (k+3/4) pi/nu (two terms of the
    // classical expansion of the zeros; relative error below 4e-7 for k >= 6),
    // as an offset from theta*_k: psi - theta*_k = pi (N - 2k - 1)/(4 N nu)
    const double psi = (k + 0.75) * pi / nu;
    double delta = pi * (double)(N - 2 * k - 1) / (4.0 * N * nu) + 1.0 / (8.0 * nu * nu * tan(psi));
    // theta*_k - pi/2 = pi (2k + 1 - N) / (2N)
    const double a0 = pi * (double)(2 * k + 1 - N) / (2.0 * N);
    const double ts = (k + 0.5) * pi / N;
    double Pv, Dv;
    node_series(P, a0, ts, delta, Pv, Dv);
    const double step = Pv / Dv;
    delta -= step;
    // 2^-54 theta is at most half an ulp of theta
    if (!__all(fabs(step) <= 0x1p-54 * (ts + delta))) {
        node_series(P, a0, ts, delta, Pv, Dv);
        delta -= Pv / Dv;
        node_series(P, a0, ts, delta, Pv, Dv);
    }
    // dP/dtheta = -(-1)^k C D;  w = 2 / (dP/dtheta)^2
    double dP = P.C * Dv;
    delta_out = delta;
    w_out = 2.0 / (dP * dP);
}

// node k (k < ceil(N/2)) and its mirror N-1-k into theta, w, dtheta
__device__ __forceinline__ void emit_node(int N, int k, double delta, double wk, double* __restrict__ theta,
                                          double* __restrict__ w, double* __restrict__ dth) {
    const double pi = 3.141592653589793;
    const double th = (k + 0.5) * pi / N + delta;
    const int k2 = N - 1 - k;
    if (theta) {
        theta[k] = th;
        if (k2 != k) theta[k2] = pi - th;
    }
    if (w) {
        w[k] = wk;
        if (k2 != k) w[k2] = wk;
    }
    if (dth) {
        dth[k] = delta;
        if (k2 != k) dth[k2] = -delta;
    }
}

// Interior nodes k >= kb, one thread each; with the closed-form boundary
// nodes (P.closed_b) also the nodes k < kb, from the plan's values.
__global__ void k_nodes_interior(NodeParams P, double* __restrict__ theta, double* __restrict__ w,
                                 double* __restrict__ dth) {
    const int N = P.N;
    const int nh = (N + 1) / 2;
    int k = (P.closed_b ? 0 : P.kb) + blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nh) return;
    double delta, wk;
    if (k < P.kb) {
        delta = P.bd[k];
        wk = P.bw[k];
    } else {
        node_interior(P, k, delta, wk);
    }
    emit_node(N, k, delta, wk, theta, w, dth);
}

// One step n -> n+1 of the Legendre recurrence in u = 2 sin^2(theta/2)
// (Reinsch's form), with r = 1/(n+1):
//   D_{n+1} = (n D_n - (2n+1) u P_n)/(n+1) = e - t - r e,  e = D_n - t, t = u P_n,
//   P_{n+1} = P_n + D_{n+1}.
__device__ __forceinline__ void reinsch_step(double u, double r, double& P, double& D) {
    double t = u * P;
    double e = D - t;
    double Dn = fma(-r, e, e - t);
    P += Dn;
    D = Dn;
}

// 1/(n+1) to full precision: hardware reciprocal plus one Newton step
__device__ __forceinline__ double recip_np1(int n) {
    double x = (double)(n + 1);
    double r = __builtin_amdgcn_rcp(x);
    r = r * fma(-x, r, 2.0);
    return fma(r, fma(-x, r, 1.0), r);
}

// Transfer data of a run of recurrence steps: the 2x2 map of the state
// (P, D) and the quadratic form Q of sum (2n+1) P_n^2 in the start state.
struct Xfer {
    double a, b, c, d;     // (P, D)_end = [[a, c], [b, d]] (P, D)_start
    double qaa, qab, qbb;  // sum = qaa P^2 + 2 qab P D + qbb D^2
};

// (first x, then y): T = Ty Tx, Q = Qx + Tx^T Qy Tx
__device__ __forceinline__ Xfer xfer_then(const Xfer& x, const Xfer& y) {
    Xfer o;
    o.a = y.a * x.a + y.c * x.b;
    o.b = y.b * x.a + y.d * x.b;
    o.c = y.a * x.c + y.c * x.d;
    o.d = y.b * x.c + y.d * x.d;
    // Tx^T Qy Tx with Tx columns (a, b) and (c, d)
    double pa = y.qaa * x.a + y.qab * x.b, pb = y.qab * x.a + y.qbb * x.b;  // Qy (a, b)
    double qa = y.qaa * x.c + y.qab * x.d, qb = y.qab * x.c + y.qbb * x.d;  // Qy (c, d)
    o.qaa = x.qaa + x.a * pa + x.b * pb;
    o.qab = x.qab + x.c * pa + x.d * pb;
    o.qbb = x.qbb + x.c * qa + x.d * qb;
    return o;
}

// P_N(cos t), P_{N-1}(cos t) and the Christoffel sum K = sum_{n<N} (2n+1) P_n^2
// for 0 < t <= pi/2: each thread of the block runs its chunk of degrees from
// the two basis states (1, 0) and (0, 1), then the chunks' transfer data are
// combined by a tree in LDS (`sh` holds 7*blockDim.x doubles, blockDim a power
// of two) and applied to the true start (P_0, D_0) = (1, 0).
__device__ void block_legendre_pair(int N, double t, double* sh, double* pN, double* pN1, double* kc) {
    const int T = blockDim.x, tid = threadIdx.x;
    double s = sin(0.5 * t);
    double u = 2.0 * s * s;
    int C = (N + T - 1) / T;
    int n0 = tid * C, n1 = min(N, n0 + C);
    double pa = 1, da = 0, pb = 0, db = 1;
    double saa = 0, sab = 0, sbb = 0;
    for (int n = n0; n < n1; ++n) {
        double wgt = 2.0 * n + 1.0;
        saa = fma(wgt * pa, pa, saa);
        sab = fma(wgt * pa, pb, sab);
        sbb = fma(wgt * pb, pb, sbb);
        double r = recip_np1(n);
        reinsch_step(u, r, pa, da);
        reinsch_step(u, r, pb, db);
    }
    Xfer x{pa, da, pb, db, saa, sab, sbb};
    for (int span = 1; span < T; span *= 2) {
        // threads tid = k*2*span hold the combined data of [k*2*span, (k*2+1)*span)
        double* q = sh + 7 * tid;
        q[0] = x.a; q[1] = x.b; q[2] = x.c; q[3] = x.d; q[4] = x.qaa; q[5] = x.qab; q[6] = x.qbb;
        __syncthreads();
        if ((tid & (2 * span - 1)) == 0 && tid + span < T) {
            const double* r = sh + 7 * (tid + span);
            Xfer y{r[0], r[1], r[2], r[3], r[4], r[5], r[6]};
            x = xfer_then(x, y);
        }
        __syncthreads();
    }
    if (tid == 0) {
        // start state (P_0, D_0) = (1, 0): P = a, D = b, K = qaa
        sh[0] = x.a;
        sh[1] = x.a - x.b;
        sh[2] = x.qaa;
    }
    __syncthreads();
    *pN = sh[0];
    *pN1 = sh[1];
    *kc = sh[2];
    __syncthreads();
}

// Boundary nodes k < kb.  The start `guess` (offset from theta*_k) is the
// Bessel-zero form theta ~ psi + (psi cot psi - 1)/(8 psi nu^2), psi =
// j_{0,k+1}/nu, nu = N + 1/2, whose error is O(nu^-4) (2.5 ulp or less from
// N = 2048 on), or theta^cheb* for small N; `newton_b` Newton steps with the
// exact recurrence follow (none for large N, where the FP64 recurrence is
// less accurate than the start).  The weight is the Christoffel number
// w_k = 2 / sum_{n<N} (2n+1) P_n(x_k)^2, which is well conditioned in x_k.
// Boundary node k: Newton steps from the start `guess0` with the exact
// recurrence (all threads of the block take part; `sh` holds 7*blockDim.x
// doubles), then the Christoffel weight.  Results valid in every thread.
__device__ void node_boundary(const NodeParams& P, double guess0, int k, double* sh, double& delta_out,
                              double& w_out) {
    const int N = P.N;
    const double pi = 3.141592653589793;
    const double ts = (k + 0.5) * pi / N;
    double delta = guess0;
    double pN, pN1, kc;
    const bool middle = (N & 1) && (k == (N - 1) / 2);
    if (middle) {
        delta = 0;  // x = 0 is a root of odd-degree P_N and theta*_k = pi/2 there
    } else {
        for (int it = 0; it < P.newton_b; ++it) {
            double th = ts + delta;
            block_legendre_pair(N, th, sh, &pN, &pN1, &kc);
            double sn, cs;
            sincos(th, &sn, &cs);
            double dP = N * (cs * pN - pN1) / sn;
            double step = pN / dP;
            delta -= step;
            if (fabs(step) <= 2.2e-16 * th) break;  // uniform across the block
        }
    }
    block_legendre_pair(N, ts + delta, sh, &pN, &pN1, &kc);
    delta_out = delta;
    w_out = 2.0 / kc;
}

// The same for one thread alone (small N): P_N, P_{N-1} and the Christoffel
// sum by the recurrence in order, Newton steps as above.
__device__ void node_boundary_thread(const NodeParams& P, double guess0, int k, double& delta_out, double& w_out) {
    const int N = P.N;
    const double pi = 3.141592653589793;
    const double ts = (k + 0.5) * pi / N;
    auto pair = [&](double t, double& pN, double& pN1, double& kc) {
        const double sh = sin(0.5 * t);
        const double u = 2.0 * sh * sh;
        double Pn = 1, Dn = 0, K = 0, Pm = 1;
        for (int n = 0; n < N; ++n) {
            K = fma((2.0 * n + 1.0) * Pn, Pn, K);
            Pm = Pn;
            reinsch_step(u, recip_np1(n), Pn, Dn);
        }
        pN = Pn;
        pN1 = Pm;
        kc = K;
    };
    double delta = guess0;
    double pN, pN1, kc;
    if ((N & 1) && (k == (N - 1) / 2)) {
        delta = 0;  // x = 0 is a root of odd-degree P_N and theta*_k = pi/2 there
    } else {
        for (int it = 0; it < P.newton_b; ++it) {
            const double th = ts + delta;
            pair(th, pN, pN1, kc);
            double sn, cs;
            sincos(th, &sn, &cs);
            const double step = pN / (N * (cs * pN - pN1) / sn);
            delta -= step;
            if (fabs(step) <= 2.2e-16 * th) break;
        }
    }
    pair(ts + delta, pN, pN1, kc);
    delta_out = delta;
    w_out = 2.0 / kc;
}

__global__ __launch_bounds__(1024) void k_nodes_boundary(NodeParams P, const double* __restrict__ guess,
                                                        double* __restrict__ theta, double* __restrict__ w,
                                                        double* __restrict__ dth) {
    extern __shared__ double sh[];
    const int k = blockIdx.x;
    double delta, wk;
    node_boundary(P, guess[k], k, sh, delta, wk);
    if (threadIdx.x == 0) emit_node(P.N, k, delta, wk, theta, w, dth);
}

// --------------------------------------------------------- ragged batches --
// Instances of uneven size N_b share one power-of-two grid of size Ng >= N_b
// (the Chebyshev points (j+1/2) pi/Ng).  Every node of P_{N_b} is paired with
// its nearest grid row j, so |Ng (theta_k - theta*_j)| <= pi/2 (for Ng = N_b
// the pairing is the identity and Lemma 2 applies).  The pairing must be
// one-to-one.  The node gaps in theta are all below pi/(N_b + 1/2) and
// smallest at the ends (Sturm comparison), where the first one is about
// 3.115/(N_b + 1/2): for N_b above about Ng/1.0085 the first few gaps are
// shorter than the grid spacing pi/Ng, so two nodes could in principle share
// a row.  They do not: there the row coordinate of node k is k plus a
// fraction that grows from about 1/4 (first node) towards 1/2 (middle), so
// node k takes row k and no rounding boundary falls between neighbours.  A
// CPU check confirms distinct rows for every such size up to Ng = 2^12 and
// for the nodes nearest the ends of sampled sizes up to 2^20.
// The Taylor series then runs about theta*_j with d = Ng (theta_k - theta*_j).
__device__ __forceinline__ int ragged_find(const int* __restrict__ off, int nb, int t) {
    int lo = 0, hi = nb;  // largest b with off[b] <= t
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void map_node(int N, int Ng, int k, double delta, double wk, int* __restrict__ gk,
                                         double* __restrict__ dg, double* __restrict__ wg) {
    const double pi = 3.141592653589793;
    for (int side = 0; side < 2; ++side) {
        const int kk = side ? N - 1 - k : k;
        if (side && kk == k) break;
        const double dd = side ? -delta : delta;
        int j = (int)rint((2.0 * kk + 1.0) * Ng / (2.0 * N) + dd * Ng / pi - 0.5);
        j = min(max(j, 0), Ng - 1);
        const int64_t I = (int64_t)(2 * kk + 1) * Ng - (int64_t)(2 * j + 1) * N;
        gk[j] = kk;
        dg[j] = Ng * dd + pi * (double)I / (2.0 * N);
        if (wg) wg[j] = wk;
    }
}

// Interior nodes of every instance, one thread each (ioff: prefix sums of
// the instances' interior node counts).  Writes the grid tables, and theta,
// w, dtheta of instance 0 when given (single non-power-of-two size).
__global__ void k_rnodes_interior(const RNode* __restrict__ R, const int* __restrict__ ioff, int nb, int Ng,
                                  int* __restrict__ gk, double* __restrict__ dg, double* __restrict__ wg,
                                  double* __restrict__ theta, double* __restrict__ w, double* __restrict__ dth) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ioff[nb]) return;
    // each instance's range starts at a multiple of 64, so a wave serves one
    // instance and its parameters are read once per wave (scalar loads)
    const int b = __builtin_amdgcn_readfirstlane(ragged_find(ioff, nb, t));
    const NodeParams& P = R[b].P;
    const int k = P.kb + (t - ioff[b]);
    if (k >= (P.N + 1) / 2) return;
    double delta, wk;
    node_interior(P, k, delta, wk);
    if (gk) map_node(P.N, Ng, k, delta, wk, gk + (int64_t)b * Ng, dg + (int64_t)b * Ng, wg ? wg + (int64_t)b * Ng : nullptr);
    if (theta || w || dth) emit_node(P.N, k, delta, wk, theta, w, dth);
}

// Boundary nodes of every instance, one block of 256 threads each (boff:
// prefix sums of the boundary node counts).
__global__ __launch_bounds__(256) void k_rnodes_boundary(const RNode* __restrict__ R, const int* __restrict__ boff,
                                                         int nb, int Ng, int* __restrict__ gk,
                                                         double* __restrict__ dg, double* __restrict__ wg,
                                                         double* __restrict__ theta, double* __restrict__ w,
                                                         double* __restrict__ dth) {
    __shared__ double sh[7 * 256];
    const int t = blockIdx.x;
    if (t >= boff[nb]) return;  // uniform per block
    const int b = ragged_find(boff, nb, t);
    const int k = t - boff[b];
    double delta, wk;
    if (R[b].P.closed_b) {  // uniform per block
        delta = R[b].P.bd[k];
        wk = R[b].P.bw[k];
    } else {
        node_boundary(R[b].P, R[b].guess[k], k, sh, delta, wk);
    }
    if (threadIdx.x == 0) {
        const int N = R[b].P.N;
        if (gk) map_node(N, Ng, k, delta, wk, gk + (int64_t)b * Ng, dg + (int64_t)b * Ng, wg ? wg + (int64_t)b * Ng : nullptr);
        if (theta || w || dth) emit_node(N, k, delta, wk, theta, w, dth);
    }
}

// Boundary nodes of every instance of a small grid, one thread each.
__global__ __launch_bounds__(256) void k_rnodes_bthread(const RNode* __restrict__ R, const int* __restrict__ boff, int nb,
                                                        int Ng, int* __restrict__ gk, double* __restrict__ dg,
                                                        double* __restrict__ wg, double* __restrict__ theta,
                                                        double* __restrict__ w, double* __restrict__ dth) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= boff[nb]) return;
    const int b = ragged_find(boff, nb, t);
    const int k = t - boff[b];
    double delta, wk;
    if (R[b].P.closed_b) {
        delta = R[b].P.bd[k];
        wk = R[b].P.bw[k];
    } else {
        node_boundary_thread(R[b].P, R[b].guess[k], k, delta, wk);
    }
    const int N = R[b].P.N;
    if (gk) map_node(N, Ng, k, delta, wk, gk + (int64_t)b * Ng, dg + (int64_t)b * Ng, wg ? wg + (int64_t)b * Ng : nullptr);
    if (theta || w || dth) emit_node(N, k, delta, wk, theta, w, dth);
}

__global__ void k_fill_int(int* __restrict__ p, int64_t n, int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// out[b*stride + n] = in[offs[b] + n] for n < N_b, 0 up to Ng (zero padding)
__global__ void k_rgather(const double* __restrict__ in, const RNode* __restrict__ R,
                          const int64_t* __restrict__ offs, int Ng, int64_t stride, double* __restrict__ out) {
    const int b = blockIdx.y;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= Ng) return;
    out[(int64_t)b * stride + n] = (n < R[b].P.N) ? in[offs[b] + n] : 0.0;
}

// out[offs[b] + n] = in[b*stride + n] for n < N_b
__global__ void k_rscatter(const double* __restrict__ in, int64_t stride, const RNode* __restrict__ R,
                           const int64_t* __restrict__ offs, double* __restrict__ out) {
    const int b = blockIdx.y;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < R[b].P.N) out[offs[b] + n] = in[(int64_t)b * stride + n];
}

// ------------------------------------------------------------------ dense --
// chat_k (k < nd) partial sums over column chunk blockIdx.y:
//   sum_{n in chunk, n >= k, n+k even} (eps_k/pi) Lam((n-k)/2) Lam((n+k)/2) c_n
// Block = 256 rows of one parity, k = kb0 + 2i + par, so every lane walks the
// same columns n (same parity); the Lam windows and c of the chunk are staged
// in LDS.  DENSE_CH columns per chunk.
constexpr int DENSE_CH = 512;

__global__ __launch_bounds__(256) void k_dense(int N, int nd, int chunk, const double* __restrict__ lam,
                                               const double* __restrict__ c, int64_t c_stride,
                                               double* __restrict__ part, int64_t part_stride) {
    __shared__ double sc[DENSE_CH], slm[DENSE_CH / 2 + 256], slp[DENSE_CH / 2 + 256];
    const int par = blockIdx.x & 1;
    const int kb0 = (blockIdx.x >> 1) * 512;
    const int ch = blockIdx.y;
    const int b = blockIdx.z;
    const double* cb = c + b * c_stride;
    double* pb = part + b * part_stride;
    const int n0 = ch * DENSE_CH, n1 = min(nd, n0 + DENSE_CH);
    const int k = kb0 + 2 * threadIdx.x + par;
    // windows: (n-k)/2 in [zm0, zm0 + CH/2 + 256), (n+k)/2 in [zp0, ...)
    const int kmax = kb0 + 511;
    const int zm0 = (n0 - kmax) >> 1;  // may be negative (unused entries)
    const int zp0 = (n0 + kb0) >> 1;
#pragma unroll
    for (int i = threadIdx.x; i < DENSE_CH; i += 256) sc[i] = (n0 + i < n1) ? cb[n0 + i] : 0.0;
#pragma unroll
    for (int i = threadIdx.x; i < DENSE_CH / 2 + 256; i += 256) {
        int zm = zm0 + i, zp = zp0 + i;
        slm[i] = (zm >= 0 && zm < nd) ? lam[zm] : 0.0;
        slp[i] = (zp >= 0 && zp < nd) ? lam[zp] : 0.0;
    }
    __syncthreads();
    if (k >= nd) return;
    int n = max(n0, k);
    if ((n - k) & 1) ++n;
    // four columns per step into four sums: the LDS reads of a step are
    // independent, so they overlap instead of each waiting for the last
    int im = ((n - k) >> 1) - zm0, ip = ((n + k) >> 1) - zp0, ic = n - n0;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (; n + 6 < n1; n += 8, im += 4, ip += 4, ic += 8) {
        a0 = fma(slm[im] * slp[ip], sc[ic], a0);
        a1 = fma(slm[im + 1] * slp[ip + 1], sc[ic + 2], a1);
        a2 = fma(slm[im + 2] * slp[ip + 2], sc[ic + 4], a2);
        a3 = fma(slm[im + 3] * slp[ip + 3], sc[ic + 6], a3);
    }
    for (; n < n1; n += 2, ++im, ++ip, ic += 2) a0 = fma(slm[im] * slp[ip], sc[ic], a0);
    const double acc = (a0 + a1) + (a2 + a3);
    double e = (k == 0) ? 0.3183098861837907 : 0.6366197723675814;  // eps_k / pi
    pb[(int64_t)ch * nd + k] = e * acc;
}

// dense[k] = sum over chunks; written to `out` (stride per instance)
__global__ void k_dense_reduce(int nd, int nchunk, int chunk, const double* __restrict__ part,
                               int64_t part_stride, double* __restrict__ out, int64_t out_stride) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.z;
    if (k >= nd) return;
    const double* pb = part + b * part_stride;
    double s = 0;
    for (int ch = k / chunk; ch < nchunk; ++ch) s += pb[(int64_t)ch * nd + k];
    out[b * out_stride + k] = s;
}

// ---------------------------------------------- batched dense block --
// The exact low block of the conversion for a batch of instances, as one
// contraction on the FP64 matrix cores.  Rows k and columns n of M pair up
// by parity p (k = 2i + p, n = 2j + p), and for each parity
//   forward:    out[b][2i+p]  = (eps_k/pi) sum_{j >= i} Lam(j-i) Lam(i+j+p) x[b][2j+p]
//   transposed: out[b][2i+p]  = h_n sum_{j <= i} Lam(i-j) Lam(i+j+p) (eps_k/pi) x[b][2j+p]
// (h_n = n + 1/2 when `half`, else 1): a Toeplitz-times-Hankel matrix that
// is the same for every instance, so each block forms its tile of it once
// (from two LDS windows of Lam) and applies it to DMM_B instances.
// Block: 4 waves; wave w takes parity w >> 1 and rows i0 + 32 (w & 1) + [0, 32)
// of tile i0 = DMM_I * blockIdx.y, instances b0 = DMM_B * blockIdx.x + [0, 32).
// Each wave accumulates a 32 x 32 tile as 2 x 2 v_mfma_f64_16x16x4f64
// (operand lanes: A row l%16, inner l/16; B column l%16, inner l/16; result
// lane l, register r -> row l/16 + 4r, column l%16), over chunks of DMM_J
// inner indices staged in LDS; each chunk's global loads are issued into
// registers while the previous chunk is multiplied.
constexpr int DMM_I = 64, DMM_B = 32, DMM_J = 64, DMM_PB = DMM_B + 4;
constexpr int DMM_XPT = 2 * DMM_J * DMM_B / 256;  // x values each thread stages per chunk
constexpr int DMM_W = DMM_I + DMM_J;              // Lam window length
typedef double dmm_v4 __attribute__((ext_vector_type(4)));

// With gridDim.z > 1 the inner range is split: block z covers the columns
// n of chunk z (DMM_CH of them) and writes its partial sums, scaled as the
// one-instance kernels' partials, at out[b * os + z * nd + k] for the
// reduction of those kernels (rows whose chunk lies wholly on the zero side
// of the triangle are neither written nor read).
constexpr int DMM_CH = DENSE_CH;  // columns per split chunk
template <bool TRANS>
__global__ __launch_bounds__(256) void k_dense_mm(int nd, const double* __restrict__ lam, const double* __restrict__ x,
                                                  int64_t xs, int nb, double* __restrict__ out, int64_t os,
                                                  int half) {
    __shared__ double sx[2 * DMM_J][DMM_PB];  // x[b0 + bb][2 j0 + t] at [t][bb]
    __shared__ double slm[DMM_W];             // Lam(|j - i|) window
    __shared__ double slp[2][DMM_W];          // Lam(i + j + p) windows
    // blocks are dispatched in x-major order: the instance tiles of one row
    // tile go together, the longest rows first (the first tiles forward,
    // the last ones transposed)
    const int ty = TRANS ? (int)(gridDim.y - 1 - blockIdx.y) : (int)blockIdx.y;
    const int i0 = ty * DMM_I, b0 = blockIdx.x * DMM_B;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int p = w >> 1, iw = i0 + 32 * (w & 1);
    const int ndp = (nd + 1 - p) >> 1;  // rows (and columns) of parity p
    const int ndp0 = (nd + 1) >> 1;
    const int lr = l & 15, lk = l >> 4;
    // inner range of the tile: forward j >= i0, transposed j <= i0 + DMM_I - 1
    int jlo = TRANS ? 0 : i0;
    int jhi = TRANS ? min(ndp0, i0 + DMM_I) : ndp0;
    const bool split = gridDim.z > 1;
    if (split) {
        const int c0 = (int)blockIdx.z * (DMM_CH / 2), c1 = c0 + DMM_CH / 2;  // chunk's inner indices
        // chunks the reduction never reads: forward, wholly left of the
        // tile's first row (c1 <= i0); transposed, wholly right of its last
        if (TRANS ? (c0 >= i0 + DMM_I) : (c1 <= i0)) return;
        jlo = max(jlo, c0);
        jhi = min(jhi, c1);
    }
    // chunk data staged through registers: the next chunk's global loads are
    // issued before the current chunk's products
    double rx[DMM_XPT], rm = 0, rp0 = 0, rp1 = 0;
    auto fetch = [&](int j0) {
#pragma unroll
        for (int e = 0; e < DMM_XPT; ++e) {
            const int q = tid + 256 * e;
            const int bb = q / (2 * DMM_J), t = q % (2 * DMM_J);
            const int n = 2 * j0 + t, b = b0 + bb;
            double v = 0.0;
            if (n < nd && b < nb) {
                v = x[(int64_t)b * xs + n];
                if (TRANS) v *= (n == 0) ? 0.3183098861837907 : 0.6366197723675814;  // eps_n / pi
            }
            rx[e] = v;
        }
        if (tid < DMM_W) {
            // forward: j - i = j0 - i0 - (DMM_I - 1) + q; transposed: i - j = i0 - j0 - (DMM_J - 1) + q
            const int zm = TRANS ? i0 - j0 - (DMM_J - 1) + tid : j0 - i0 - (DMM_I - 1) + tid;
            rm = (zm >= 0 && zm < nd) ? lam[zm] : 0.0;
            const int zp = i0 + j0 + tid;
            rp0 = (zp < nd) ? lam[zp] : 0.0;
            rp1 = (zp + 1 < nd) ? lam[zp + 1] : 0.0;
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int e = 0; e < DMM_XPT; ++e) {
            const int q = tid + 256 * e;
            sx[q % (2 * DMM_J)][q / (2 * DMM_J)] = rx[e];
        }
        if (tid < DMM_W) {
            slm[tid] = rm;
            slp[0][tid] = rp0;
            slp[1][tid] = rp1;
        }
    };
    dmm_v4 acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[u][t] = dmm_v4{0, 0, 0, 0};
    if (jlo < jhi) fetch(jlo);
    for (int j0 = jlo; j0 < jhi; j0 += DMM_J) {
        __syncthreads();  // the previous chunk's reads are done
        stage();
        __syncthreads();
        if (j0 + DMM_J < jhi) fetch(j0 + DMM_J);
#pragma unroll 4
        for (int s4 = 0; s4 < DMM_J; s4 += 4) {
            const int jj = s4 + lk;  // inner index within the chunk
            double a[2], bv[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int ii = iw - i0 + 16 * u + lr;  // row within the tile
                const double lm = TRANS ? slm[ii - jj + (DMM_J - 1)] : slm[jj - ii + (DMM_I - 1)];
                a[u] = lm * slp[p][ii + jj];
            }
#pragma unroll
            for (int t = 0; t < 2; ++t) bv[t] = sx[2 * jj + p][16 * t + lr];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int t = 0; t < 2; ++t) acc[u][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bv[t], acc[u][t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = iw + 16 * u + lk + 4 * r, b = b0 + 16 * t + lr;
                if (i < ndp && b < nb) {
                    const int k = 2 * i + p;
                    const double sc = TRANS ? ((half && !split) ? k + 0.5 : 1.0)
                                            : ((k == 0) ? 0.3183098861837907 : 0.6366197723675814);
                    out[(int64_t)b * os + (split ? (int64_t)blockIdx.z * nd : 0) + k] = sc * acc[u][t][r];
                }
            }
}

// ------------------------------------------------------ FFT pass helpers --
// Every FFT-carrying kernel: FFT_THREADS threads, and registers capped so that
// FFT_WAVES waves of it share a SIMD (the LDS tile allows three blocks per CU)
#ifndef FFT_WAVES
#define FFT_WAVES 2
#endif
#define FFT_BOUNDS __launch_bounds__(FFT_THREADS) __attribute__((amdgpu_waves_per_eu(FFT_WAVES)))
// the same for a kernel whose FP32 tiles (half the LDS) of compile-time
// length L fit the registers of three waves per SIMD without spilling (the
// FP32 passes A of the far field and of the Taylor terms, both directions,
// and the FP32 Taylor pass B)
#define FFT_BOUNDS_R(R, L) \
    __launch_bounds__(FFT_THREADS) __attribute__((amdgpu_waves_per_eu((sizeof(R) == 4 && (L) > 0) ? 3 : FFT_WAVES)))
// Intermediate layout between the passes ("blocked"): DFT output (n_a, j_b)
// of pass A sits at X[(v >> lrB) * (N1 << lrB) + n_a * rowsB + (v & (rowsB-1))]
// with v = j_b, or for kernels whose pass B pairs row r with N2 - r, the
// virtual row v(j_b) that places the pair next to each other:
// v(0) = 0, v(N2/2) = 1, v(r) = 2r, v(N2-r) = 2r+1 (0 < r < N2/2).
// A pass-B tile of rowsB (virtual) rows is one contiguous block.
__device__ __forceinline__ int virt_row(int jb, int N2) {
    if (N2 <= 2) return jb;
    if (jb == 0) return 0;
    if (jb == N2 / 2) return 1;
    return (jb < N2 / 2) ? 2 * jb : 2 * (N2 - jb) + 1;
}
__device__ __forceinline__ int actual_row(int v, int N2) {
    if (N2 <= 2) return v;
    if (v == 1) return N2 / 2;
    return (v & 1) ? N2 - (v >> 1) : (v >> 1);
}

// blocks are dispatched round-robin to the 8 XCDs; give each XCD a
// contiguous range of tiles so neighbouring tiles share an L2
__device__ __forceinline__ int xcd_tile(int bid, int ntiles) {
    if (ntiles & 7) return bid;
    return (bid & 7) * (ntiles >> 3) + (bid >> 3);
}
// the same with each XCD's range split into a run from the front and its
// mirror image from the back (tiles t and ntiles - 1 - t on one XCD): the
// passes that store or load vectors in grid-row order (rows 2m and 2m + 1
// come from the tiles of m and N - 1 - m, which are mirror tiles) then
// complete or consume each line in one L2
__device__ __forceinline__ int xcd_tile_mirror(int bid, int ntiles) {
    if (ntiles & 15) return xcd_tile(bid, ntiles);
    const int half = ntiles >> 4, x = bid & 7, k = bid >> 3;
    return (k < half) ? x * half + k : ntiles - 1 - (x * half + (k - half));
}

// Pass A: the block owns columns n_a in [na0, na0+colsA) and runs the
// length-N2 DFTs over n_b (element (col, idx) of the tile is n_a = na0 + col,
// n_b = idx, input index n = n_a + N1 n_b).  Output j_b = idx of the same
// element is multiplied by e^{2 pi i n_a j_b / N} and stored in the blocked
// layout.  With a compile-time length the thread's column is fixed and its
// j_b are i0 + s L/8, so the twiddles are e^{2 pi i n_a i0/N} times powers
// of e^{2 pi i n_a L/(8N)}, kept as that start value and the 1st, 2nd and 4th
// powers (every twiddle is at most three products away from table values).
__device__ __forceinline__ int passA_offset(const Geo& g, int na, int jb, bool virt) {
    const int vr = virt ? virt_row(jb, g.N2) : jb;
    return (vr >> g.lrB) * (g.N1 << g.lrB) + na * g.rowsB + (vr & (g.rowsB - 1));
}

template <int L, bool VIRT>
struct PassAOut {
    cplx w0, p1, p2, p4;
    int na;
    __device__ __forceinline__ PassAOut(const Geo& g, const Tile<L>& T, int na0) {
        na = na0 + T.col(0);
        w0 = tw2(g.twHi, g.twLo, (int64_t)na * T.idx(0), g.sh);
        p1 = tw2(g.twHi, g.twLo, (int64_t)na * (L / 8), g.sh);
        p2 = tw2(g.twHi, g.twLo, (int64_t)na * (L / 4), g.sh);
        p4 = tw2(g.twHi, g.twLo, (int64_t)na * (L / 2), g.sh);
    }
    // the thread's twiddles w[s] (element s)
    __device__ __forceinline__ void twiddles(cplx* w) const {
        w[0] = w0;
        w[1] = cmul(w0, p1);
        w[2] = cmul(w0, p2);
        w[3] = cmul(w[1], p2);
        w[4] = cmul(w0, p4);
        w[5] = cmul(w[1], p4);
        w[6] = cmul(w[2], p4);
        w[7] = cmul(w[3], p4);
    }
    // o[s] = v[s] times its twiddle
    template <class R>
    __device__ __forceinline__ void twid(const cplxT<R>* v, cplxT<R>* o) const {
        cplx w[8];
        twiddles(w);
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) o[s] = cto<R>(cmul(cwide(v[s]), w[s]));
    }
    // stores the twiddled element s
    template <class R>
    __device__ __forceinline__ void store(const Geo& g, const cplxT<R>* o, cplxT<R>* __restrict__ Xt,
                                          const Tile<L>& T, int s) const {
        Xt[passA_offset(g, na, T.idx(s), VIRT)] = o[s];
    }
    template <class R>
    __device__ __forceinline__ void put(const Geo& g, const cplxT<R>* v, cplxT<R>* __restrict__ Xt,
                                        const Tile<L>& T) const {
        cplxT<R> o[FFT_VPT];
        twid(v, o);
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) store(g, o, Xt, T, s);
    }
};

template <bool VIRT>
struct PassAOut<0, VIRT> {
    cplx w[FFT_VPT];
    int na0;
    __device__ __forceinline__ PassAOut(const Geo& g, const Tile<0>& T, int na0_) : na0(na0_) {
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s)
            if (T.live(s)) w[s] = tw2(g.twHi, g.twLo, (int64_t)(na0 + T.col(s)) * T.idx(s), g.sh);
    }
    template <class R>
    __device__ __forceinline__ void twid(const cplxT<R>* v, cplxT<R>* o) const {
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) o[s] = cto<R>(cmul(cwide(v[s]), w[s]));
    }
    template <class R>
    __device__ __forceinline__ void store(const Geo& g, const cplxT<R>* o, cplxT<R>* __restrict__ Xt,
                                          const Tile<0>& T, int s) const {
        if (T.live(s)) Xt[passA_offset(g, na0 + T.col(s), T.idx(s), VIRT)] = o[s];
    }
    template <class R>
    __device__ __forceinline__ void put(const Geo& g, const cplxT<R>* v, cplxT<R>* __restrict__ Xt,
                                        const Tile<0>& T) const {
        cplxT<R> o[FFT_VPT];
        twid(v, o);
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) store(g, o, Xt, T, s);
    }
};

// Pass-A output of one tile held back and stored during the transform of the
// block's next tile, a few stores after each of its LDS exchanges: the stores
// of a term then stream out while the next term is transformed, instead of
// leaving in one burst between two transforms.
template <int L, bool VIRT, class R>
struct HeldPut {
    // FP32 tiles of compile-time length: the thread's twiddles are rounded
    // to FP32 once and applied in FP32 (the FP32 terms' own rounding is of
    // that order), instead of widening every product to FP64
    static constexpr bool F32 = (sizeof(R) < sizeof(double)) && (L > 0);
    const PassAOut<L, VIRT>& out;
    const Geo& g;
    const Tile<L>& T;
    cplxT<R> o[FFT_VPT];
    cplxT<R> wr[F32 ? FFT_VPT : 1];
    cplxT<R>* dst = nullptr;
    __device__ __forceinline__ HeldPut(const PassAOut<L, VIRT>& out_, const Geo& g_, const Tile<L>& T_)
        : out(out_), g(g_), T(T_) {
        if constexpr (F32) {
            cplx w[FFT_VPT];
            out.twiddles(w);
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) wr[s] = cto<R>(w[s]);
        }
    }
    // stores the held tile's share of hook point pt (none before the first hold)
    __device__ __forceinline__ void operator()(int pt) const {
        constexpr int NP = tile_hook_points<L>();
        if (dst) {
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s)
                if (s * NP / FFT_VPT == pt) out.store(g, o, dst, T, s);
        }
    }
    // holds the transform v, bound for the slab Xt
    __device__ __forceinline__ void hold(const cplxT<R>* v, cplxT<R>* Xt) {
        if constexpr (F32) {
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) o[s] = cmul(v[s], wr[s]);
        } else {
            out.twid(v, o);
        }
        dst = Xt;
    }
    // twiddles the transform v and stores it at once (nothing is held)
    __device__ __forceinline__ void put(const cplxT<R>* v, cplxT<R>* Xt) const {
        cplxT<R> t[FFT_VPT];
        if constexpr (F32) {
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) t[s] = cmul(v[s], wr[s]);
        } else {
            out.twid(v, t);
        }
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) out.store(g, t, Xt, T, s);
    }
    __device__ __forceinline__ void flush() {
        if (dst) {
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) out.store(g, o, dst, T, s);
        }
        dst = nullptr;
    }
};

// Pass B: the block owns (virtual) rows [vb0, vb0+rowsB) of the blocked
// intermediate, one contiguous run of rowsB*N1 values in which element
// (row, n_a) = (col, idx) of the tile sits at n_a*rowsB + row, which is
// thread + s*FFT_THREADS for the thread's element s.  After the length-N1 DFTs
// element (row, j_a) is output m = jb(row) + N2 j_a.
template <int L, class R>
__device__ __forceinline__ void passB_load(const Geo& g, int vb0, const cplxT<R>* __restrict__ X, cplxT<R>* v,
                                           const Tile<L>& T) {
    const cplxT<R>* src = X + (int64_t)(vb0 >> g.lrB) * ((int64_t)g.N1 << g.lrB);
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s)
        if (T.live(s)) v[s] = src[threadIdx.x + s * FFT_THREADS];
}

// The far-field term list, entry l in lane l (MAX_TERMS = wave size): the
// loops over terms take a term's fields with readlane, a register operation,
// instead of a scalar load from the kernel arguments and its wait (which also
// drains the outstanding LDS operations) in every iteration.
static_assert(MAX_TERMS <= 64, "one term per lane");
struct FarTerms {
    int m_, blk_, nlo_;
    __device__ __forceinline__ explicit FarTerms(const FarParams& F) {
        const int l = (int)threadIdx.x & 63;
        const bool in = l < F.nterm;
        m_ = in ? F.term_m[l] : 0;
        blk_ = in ? F.term_blk[l] : 0;
        nlo_ = in ? F.blk[blk_].nlo : 0;
    }
    __device__ __forceinline__ int m(int t) const { return __builtin_amdgcn_readlane(m_, t); }
    __device__ __forceinline__ int blk(int t) const { return __builtin_amdgcn_readlane(blk_, t); }
    __device__ __forceinline__ int nlo(int t) const { return __builtin_amdgcn_readlane(nlo_, t); }
};

// ---------------------------------------------------------- far field A --
// Terms t are ordered by ascending m.  For every term, taken in descending m
// so that h_{m-1,n} = h_{m,n} m (n+m+1/2)/(m-1/2)^2 needs no division, the
// DFT input
//   b_n = C_n h_{m,n} c_n e^{i pi n/(2N)} [n >= nlo_b]
// goes through pass A of the length-N DFT.  Term group blockIdx.y takes the
// terms nterm-1-y, nterm-1-y-G, ...
template <int LA, class R>
__global__ FFT_BOUNDS_R(R, LA) void k_far_passA(Geo g, FarParams F, int G, const cplx* __restrict__ amp,
                                                          const double* __restrict__ c, int64_t c_stride,
                                                          cplxT<R>* __restrict__ X, int64_t x_stride) {
    // FP32 tiles are transformed in pairs of terms (two tiles); FP64 tiles
    // one at a time (a pair would not fit the registers of two waves per SIMD)
    constexpr bool PAIRS = sizeof(R) == sizeof(float);
    __shared__ cplxT<R> buf[TILE_LDS(LA) * (PAIRS ? 2 : 1)];
    cplxT<R>* const buf2 = buf + TILE_LDS(LA);
    STAGE_TW(stw, LA, R);
    const cplxT<R>* twA = stage_twiddles<LA, R>(stw, g.twN2, g.N2);
    const Tile<LA> T(g.colsA, g.N2);
    const FarTerms FT(F);
    const int N = g.N;
    const int na0 = xcd_tile(blockIdx.x, gridDim.x) * T.cols();
    const int b = blockIdx.z;
    const double* cb = c + b * c_stride;
    cplxT<R>* Xb = X + b * x_stride;
    const PassAOut<LA, false> out(g, T, na0);
    // C_n h_{m,n} c_n e^{i pi n/(2N)} at the current m, carried in the
    // precision of the terms (FP32 terms: its FP32 rounding per step is that
    // of the terms themselves)
    using BT = typename std::conditional<PAIRS, R, double>::type;
    cplxT<BT> bh[FFT_VPT];
    int nn[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        bh[s] = {0, 0};
        nn[s] = -1;
        if (T.live(s)) {
            const int n = na0 + T.col(s) + g.N1 * T.idx(s);
            nn[s] = n;
            if (n >= F.nd) bh[s] = cto<BT>(cscale(amp[n], cb[n]));
        }
    }
    int mcur = F.Mmax - 1;
    // the input of term t at the current m (advanced down to term t's m)
    auto input = [&](int t, cplxT<R>* v) {
        const int m = FT.m(t);
        for (; mcur > m; --mcur) {
            const double fm = (double)mcur / ((mcur - 0.5) * (mcur - 0.5));
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) bh[s] = cscale(bh[s], (BT)(fm * (nn[s] + mcur + 0.5)));
        }
        const int nlo = FT.nlo(t);
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            if constexpr (PAIRS) v[s] = (nn[s] >= nlo) ? bh[s] : cplxT<R>{0, 0};
            else v[s] = (nn[s] >= nlo) ? cto<R>(bh[s]) : cplxT<R>{0, 0};
        }
    };
    // terms in pairs (t, t - G): two tiles per barrier sequence
    int t = F.nterm - 1 - (int)blockIdx.y;
    HeldPut<LA, false, R> held(out, g, T);
    if constexpr (PAIRS) {
        for (; t - G >= 0; t -= 2 * G) {
            cplxT<R> v1[FFT_VPT], v2[FFT_VPT];
            input(t, v1);
            input(t - G, v2);
            tile_fft2<LA>(v1, v2, buf, buf2, twA, T);
            held.put(v1, Xb + (int64_t)t * N);
            held.put(v2, Xb + (int64_t)(t - G) * N);
        }
    }
    for (; t >= 0; t -= G) {
        cplxT<R> v[FFT_VPT];
        input(t, v);
        tile_fft<LA>(v, buf, twA, T, held);
        held.hold(v, Xb + (int64_t)t * N);
    }
    held.flush();
}

// ---------------------------------------------------------- far field B --
// For every term the z-values z_j = sum_n b_n e^{i n theta_j} (z = V_m or
// conj(V_m) at row j(m)) are combined into
//   v_j += Re(e^{i (m+1/2)(theta_j - pi/2)} z_j) / (2 sin theta_j)^{m+1/2}
// on the rows of the term's block.  Term group blockIdx.y handles terms
// t = y, y + G, ... (ascending m); partial values go to v[y].  The next
// term's tile is loaded while the current one is transformed.
__device__ __forceinline__ int row_block(const FarParams& F, int j, int N) {
    int jj = min(j, N - 1 - j);
    for (int b = 0; b < F.nblk; ++b)
        if (jj >= F.blk[b].jlo && jj < F.blk[b].jhi) return b;
    return -1;
}

// e^{i (theta_j - pi/2)/2} (2 sin theta_j)^{-1/2} and e^{i (theta_j - pi/2)} / (2 sin theta_j)
__device__ __forceinline__ void far_row_factors(int j, int N, cplx& g0, cplx& rq) {
    const double pi = 3.141592653589793;
    double d = pi * (double)(2 * j + 1 - N) / (2.0 * N);  // theta_j - pi/2
    int jj = min(j, N - 1 - j);
    double sn = sin((jj + 0.5) * pi / N);                 // sin theta_j, full relative accuracy
    double q = 1.0 / (2.0 * sn);
    double ps, pc, rs, rc;
    sincos(0.5 * d, &ps, &pc);
    sincos(d, &rs, &rc);
    double r0 = sqrt(q);
    g0 = {pc * r0, ps * r0};
    rq = {rc * q, rs * q};
}

// Plan time: the far-field tables (see Plan::d_amp, Plan::d_rowf), one
// thread per index.
__global__ void k_far_tables(int N, FarParams F, cplx* __restrict__ amp, cplx* __restrict__ rowf) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    cplx a = {0, 0};
    if (n >= F.nd) {
        // h_{Mmax-1,n} = K / prod_{j<Mmax} (n+j+1/2),  K = prod_{j<Mmax} (j-1/2)^2/j
        double den = 1;
        for (int j = 1; j < F.Mmax; ++j) den *= (n + j + 0.5);
        a = cscale(half_shift(n, N), stieltjes_C((double)n) * (F.hK / den));
    }
    amp[n] = a;
    // row factor by DFT output index m = n (row j(m)), the order in which
    // the passes read it; the ratio between consecutive m is its square
    cplx g0, rq;
    far_row_factors(row_of(n, N), N, g0, rq);
    rowf[n] = g0;
}

template <int LB, class R>
__global__ FFT_BOUNDS void k_far_passB(Geo g, FarParams F, int G, const cplx* __restrict__ rowf,
                                                          const cplxT<R>* __restrict__ X, int64_t x_stride,
                                                          double* __restrict__ v, int64_t v_stride) {
    __shared__ cplxT<R> buf[TILE_LDS(LB)];
    STAGE_TW(stw, LB, R);
    const cplxT<R>* twB = stage_twiddles<LB, R>(stw, g.twN1, g.N1);
    const Tile<LB> T(g.rowsB, g.N1);
    const FarTerms FT(F);
    const int N = g.N;
    const int jb0 = xcd_tile_mirror(blockIdx.x, gridDim.x) * T.cols();
    const int grp = blockIdx.y;
    const int b = blockIdx.z;
    const cplxT<R>* Xb = X + b * x_stride;
    cplx gm[FFT_VPT], rq[FFT_VPT];
    double acc[FFT_VPT];
    int key[FFT_VPT];  // 2 * block + (conjugated output), -1 outside
    int t = grp;
    // the first tile's loads go out before the row factors', so that
    // waiting for the tile does not wait for the factors (loads retire in
    // order)
    cplxT<R> nx[FFT_VPT] = {};
    if (t < F.nterm) passB_load<LB, R>(g, jb0, Xb + (int64_t)t * N, nx, T);
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        acc[s] = 0;
        key[s] = -1;
        gm[s] = {0, 0};
        if (T.live(s)) {
            const int mo = jb0 + T.col(s) + g.N2 * T.idx(s);
            const int j = row_of(mo, N);
            const int blk = row_block(F, j, N);
            if (blk >= 0) key[s] = 2 * blk + (2 * mo >= N ? 1 : 0);
            gm[s] = rowf[mo];
        }
    }
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) rq[s] = cmul(gm[s], gm[s]);
    int mcur = 0;
    for (; t < F.nterm; t += G) {
        const int m = FT.m(t);
        const int tb = FT.blk(t);
        cplxT<R> z[FFT_VPT];
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) z[s] = nx[s];
        if (t + G < F.nterm) passB_load<LB, R>(g, jb0, Xb + (int64_t)(t + G) * N, nx, T);
        for (; mcur < m; ++mcur) {
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) gm[s] = cmul(gm[s], rq[s]);
        }
        tile_fft<LB>(z, buf, twB, T);
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            if ((key[s] >> 1) == tb) {
                const double zr = (double)z[s].re, zi = (key[s] & 1) ? -(double)z[s].im : (double)z[s].im;
                acc[s] = fma(gm[s].re, zr, fma(-gm[s].im, zi, acc[s]));
            }
        }
    }
    double* vb = v + b * v_stride + (int64_t)grp * N;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        if (T.live(s)) {
            const int mo = jb0 + T.col(s) + g.N2 * T.idx(s);
            vb[row_of(mo, N)] = acc[s];
        }
    }
}

// ------------------------------------------------------------ near field --
// Rows j < jnear (and their mirrors N-1-j) take the direct recurrence over
// degrees [nd, nend) of their segment, split into chunks of NEAR_CHUNK
// degrees.  Work-group = one wave = 64 consecutive rows of one segment and
// one chunk; the plan's table maps blockIdx.x to (segment, chunk, row group).
// Degrees and 1/(n+1) are uniform across the wave.
struct NearWG {
    int seg, ch, grp;
};

__device__ __forceinline__ NearWG near_wg(const NearParams& NP, const int* __restrict__ wg_seg,
                                          const int* __restrict__ segoff, int wgid) {
    NearWG w;
    w.seg = wg_seg[wgid];
    const Seg& S = NP.seg[w.seg];
    int ng = (S.jhi - S.jlo + 63) >> 6;
    int loc = wgid - segoff[2 * w.seg];
    w.ch = loc / ng;
    w.grp = loc - w.ch * ng;
    return w;
}

// Transfer data of item (row, chunk), used once per plan: for chunk 0 the
// state (P, D) at its end from the true start (P_0, D_0) = (1, 0); for later
// chunks the images of the basis states (1, 0) and (0, 1), i.e. the chunk's
// 2x2 transfer matrix.  Item record: 8 doubles (end state | matrix).
__global__ __launch_bounds__(64) void k_near_items(int N, NearParams NP, const int* __restrict__ wg_seg,
                                                   const int* __restrict__ segoff, const double* __restrict__ rcp,
                                                   double* __restrict__ items) {
    const NearWG W = near_wg(NP, wg_seg, segoff, blockIdx.x);
    const Seg S = NP.seg[W.seg];
    const int nrows = S.jhi - S.jlo;
    const int row = W.grp * 64 + threadIdx.x;
    const bool act = row < nrows;
    const int j = S.jlo + (act ? row : nrows - 1);
    const double pi = 3.141592653589793;
    double sn = sin(0.5 * (j + 0.5) * pi / N);
    const double u = 2.0 * sn * sn;
    const int n0 = W.ch * NEAR_CHUNK, n1 = min(S.nend, n0 + NEAR_CHUNK);
    double* out = items + (int64_t)(S.item_off + W.ch * nrows + row) * 8;
    if (W.ch == 0) {
        double p = 1, d = 0;
        for (int n = n0; n < n1; ++n) reinsch_step(u, rcp[n], p, d);
        if (act) {
            out[0] = p;
            out[1] = d;
        }
    } else {
        double pa = 1, da = 0, pb = 0, db = 1;
        for (int n = n0; n < n1; ++n) {
            double r = rcp[n];
            reinsch_step(u, r, pa, da);
            reinsch_step(u, r, pb, db);
        }
        if (act) {
            out[0] = pa;
            out[1] = da;
            out[2] = pb;
            out[3] = db;
        }
    }
}

// Plan time: from the state at each chunk start (2 doubles per item), the
// states every NEAR_SUB degrees inside the chunk (2 * NEAR_NSUB per item).
// The recurrence may run past the segment's last degree; such states are
// never weighted.
__global__ __launch_bounds__(64) void k_near_substates(int N, NearParams NP, const int* __restrict__ wg_seg,
                                                       const int* __restrict__ segoff,
                                                       const double* __restrict__ rcp,
                                                       const double* __restrict__ st1, double* __restrict__ st) {
    const NearWG W = near_wg(NP, wg_seg, segoff, blockIdx.x);
    const Seg S = NP.seg[W.seg];
    const int nrows = S.jhi - S.jlo;
    const int row = W.grp * 64 + threadIdx.x;
    if (row >= nrows) return;
    const int j = S.jlo + row;
    const double pi = 3.141592653589793;
    const double sn = sin(0.5 * (j + 0.5) * pi / N);
    const double u = 2.0 * sn * sn;
    const int id = S.item_off + W.ch * nrows + row;
    double p = st1[2 * id], d = st1[2 * id + 1];
    const int n0 = W.ch * NEAR_CHUNK;
    for (int k = 0; k < NEAR_NSUB; ++k) {
        st[(int64_t)id * 2 * NEAR_NSUB + 2 * k] = p;
        st[(int64_t)id * 2 * NEAR_NSUB + 2 * k + 1] = d;
        if (k + 1 < NEAR_NSUB)
            for (int n = n0 + k * NEAR_SUB; n < n0 + (k + 1) * NEAR_SUB; ++n) reinsch_step(u, rcp[n], p, d);
    }
}

// Forward near field from the plan's states: work-group = 64 consecutive
// rows of one segment and one degree chunk [n0, n1); each lane runs the
// NEAR_NSUB sub-chunks of its row as independent recurrences (from the
// stored states) side by side and forms
//   E = sum_{n even, n >= nd} c_n P_n(x_j),  O = sum_{n odd, n >= nd} c_n P_n(x_j)
// over the chunk.  Chunks that end at or below nd have nothing to add.
__global__ __launch_bounds__(64) void k_near_sums(int N, NearParams NP, const int* __restrict__ wg_seg,
                                                  const int* __restrict__ segoff, const double* __restrict__ rcp,
                                                  const double* __restrict__ st, const double* __restrict__ c,
                                                  int64_t c_stride, double* __restrict__ sums, int64_t s_stride) {
    const NearWG W = near_wg(NP, wg_seg, segoff, blockIdx.x);
    const Seg S = NP.seg[W.seg];
    const int n0 = W.ch * NEAR_CHUNK, n1 = min(S.nend, n0 + NEAR_CHUNK);
    if (n1 <= NP.nd) return;
    const int b = blockIdx.z;
    const int nrows = S.jhi - S.jlo;
    const int row = W.grp * 64 + threadIdx.x;
    const bool act = row < nrows;
    const int rr = act ? row : nrows - 1;
    const int j = S.jlo + rr;
    const double pi = 3.141592653589793;
    const double sn = sin(0.5 * (j + 0.5) * pi / N);
    const double u = 2.0 * sn * sn;
    const int id = S.item_off + W.ch * nrows + rr;
    // the chunk's 1/(n+1) and c_n (zero below nd and from n1 on) in LDS;
    // the recurrences run the whole chunk (rcp covers n < N, a multiple of
    // NEAR_CHUNK)
    __shared__ double sr[NEAR_CHUNK], sc[NEAR_CHUNK];
    const double* cb = c + b * c_stride;
    {
        // all loads first, then the LDS stores
        double lr[NEAR_CHUNK / 64], lc[NEAR_CHUNK / 64];
#pragma unroll
        for (int q = 0; q < NEAR_CHUNK / 64; ++q) {
            const int n = n0 + (int)threadIdx.x + 64 * q;
            lr[q] = rcp[n];
            lc[q] = (n >= NP.nd && n < n1) ? cb[n] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NEAR_CHUNK / 64; ++q) {
            sr[threadIdx.x + 64 * q] = lr[q];
            sc[threadIdx.x + 64 * q] = lc[q];
        }
    }
    __syncthreads();
    double p[NEAR_NSUB], d[NEAR_NSUB], E[NEAR_NSUB], O[NEAR_NSUB];
#pragma unroll
    for (int k = 0; k < NEAR_NSUB; ++k) {
        p[k] = st[(int64_t)id * 2 * NEAR_NSUB + 2 * k];
        d[k] = st[(int64_t)id * 2 * NEAR_NSUB + 2 * k + 1];
        E[k] = O[k] = 0;
    }
    // sub-chunk starts are even, so even offsets are even degrees
#pragma unroll 2
    for (int i = 0; i < NEAR_SUB; i += 2) {
#pragma unroll
        for (int k = 0; k < NEAR_NSUB; ++k) {
            const int o = k * NEAR_SUB + i;
            E[k] = fma(sc[o], p[k], E[k]);
            reinsch_step(u, sr[o], p[k], d[k]);
            O[k] = fma(sc[o + 1], p[k], O[k]);
            reinsch_step(u, sr[o + 1], p[k], d[k]);
        }
    }
    if (act) {
        double Es = 0, Os = 0;
#pragma unroll
        for (int k = 0; k < NEAR_NSUB; ++k) {
            Es += E[k];
            Os += O[k];
        }
        double* o = sums + b * s_stride + 2 * (int64_t)id;
        o[0] = Es;
        o[1] = Os;
    }
}

// One wave per endpoint row j < jnear: sums the chunk results of the row;
// near[j] = E + O (row j), near[jnear + j] = E - O (row N-1-j), since
// P_n(-x) = (-1)^n P_n(x).
__global__ __launch_bounds__(64) void k_near_reduce(NearParams NP, const double* __restrict__ sums,
                                                    int64_t s_stride, double* __restrict__ near,
                                                    int64_t near_stride) {
    const int j = blockIdx.x;
    const int b = blockIdx.z;
    const int lane = threadIdx.x;
    double E = 0, O = 0;
    int sgi = -1;
    for (int q = 0; q < NP.nseg; ++q)
        if (j >= NP.seg[q].jlo && j < NP.seg[q].jhi) sgi = q;
    if (sgi >= 0) {
        const Seg S = NP.seg[sgi];
        const int nrows = S.jhi - S.jlo;
        const int id0 = S.item_off + (j - S.jlo);
        const double* sb = sums + b * s_stride;
        for (int ch = NP.nd / NEAR_CHUNK + lane; ch < S.nchunk; ch += 64) {
            const double* o = sb + 2 * (int64_t)(id0 + ch * nrows);
            E += o[0];
            O += o[1];
        }
    }
    for (int k = 32; k >= 1; k >>= 1) {
        E += __shfl_xor(E, k);
        O += __shfl_xor(O, k);
    }
    if (lane == 0) {
        double* nb = near + b * near_stride;
        nb[j] = E + O;
        nb[NP.jnear + j] = E - O;
    }
}

__device__ __forceinline__ int near_seg_of(const NearParams& NP, int j) {
    int sgi = -1;
    for (int s = 0; s < NP.nseg; ++s)
        if (j >= NP.seg[s].jlo && j < NP.seg[s].jhi) sgi = s;
    return sgi;
}

// ----------------------------------------------------------------- DCT-II --
// chat_n = (eps_n/N) sum_j v_j cos(n theta_j) + dense_n:  DFT of
// p_m = v_{j(m)}, then chat_n = (eps_n/N) Re(e^{i pi n/(2N)} U_n).
// v_j is the sum of the G far-field partials and the near-field value.
template <int LA>
__global__ FFT_BOUNDS void k_dct2_passA(Geo g, int G, const double* __restrict__ v,
                                                           int64_t v_stride, const double* __restrict__ near,
                                                           int64_t near_stride, int jnear, cplx* __restrict__ X,
                                                           int64_t x_stride) {
    __shared__ cplx buf[TILE_LDS(LA)];
    STAGE_TW(stw, LA, double);
    const cplx* twA = stage_twiddles<LA, double>(stw, g.twN2, g.N2);
    const Tile<LA> T(g.colsA, g.N2);
    const int N = g.N;
    const int na0 = xcd_tile_mirror(blockIdx.x, gridDim.x) * T.cols();
    const int b = blockIdx.z;
    const double* vb = v + b * v_stride;
    const double* nb = near + b * near_stride;
    const PassAOut<LA, false> out(g, T, na0);
    cplx x[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        if (T.live(s)) {
            const int m = na0 + T.col(s) + g.N1 * T.idx(s);
            const int j = row_of(m, N);
            double a = 0;
            for (int q = 0; q < G; ++q) a += vb[(int64_t)q * N + j];
            if (j < jnear) a += nb[j];
            else if (N - 1 - j < jnear) a += nb[jnear + (N - 1 - j)];
            x[s] = {a, 0.0};
        }
    }
    tile_fft<LA>(x, buf, twA, T);
    out.put(g, x, X + b * x_stride, T);
}

template <int LB>
__global__ FFT_BOUNDS void k_dct2_passB(Geo g, int nd, const cplx* __restrict__ X,
                                                           int64_t x_stride, const double* __restrict__ dense,
                                                           int64_t dense_stride, double* __restrict__ chat,
                                                           int64_t chat_stride) {
    __shared__ cplx buf[TILE_LDS(LB)];
    STAGE_TW(stw, LB, double);
    const cplx* twB = stage_twiddles<LB, double>(stw, g.twN1, g.N1);
    const Tile<LB> T(g.rowsB, g.N1);
    const int N = g.N;
    const int jb0 = xcd_tile(blockIdx.x, gridDim.x) * T.cols();
    const int b = blockIdx.z;
    cplx z[FFT_VPT];
    passB_load<LB, double>(g, jb0, X + b * x_stride, z, T);
    cplx eh[FFT_VPT];  // e^{i pi n/(2N)} of the thread's elements
    if constexpr (LB > 0) half_shift_eighths(g, jb0 + T.col(0) + g.N2 * T.idx(0), eh);
    tile_fft<LB>(z, buf, twB, T);
    const double* db = dense + b * dense_stride;
    double* cb = chat + b * chat_stride;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        if (T.live(s)) {
            const int n = jb0 + T.col(s) + g.N2 * T.idx(s);
            const cplx t = (LB > 0) ? eh[s] : half_shift_tab(g, n);
            double val = (t.re * z[s].re - t.im * z[s].im) * ((n == 0) ? 1.0 : 2.0) / N;
            if (n < nd) val += db[n];
            cb[n] = val;
        }
    }
}

// ------------------------------------------------------------------ NDCT --
// Pair q of Taylor terms (l = 2q: cosine sum of (n/N)^{2q} chat, l = 2q+1:
// sine sum of (n/N)^{2q+1} chat) as one DFT of the Hermitian-split input
//   W_n = (e^{i pi n/(2N)}/2) [x^{2q}(1+x) chat_n - i y^{2q} x chat_{N-n}],
// x = n/N, y = 1 - x (n >= 1), W_0 = chat_0 [q = 0]; then at output m the
// cosine term is Re U_m and the sine term sigma_m Im U_m, row k = j(m).
// One launch covers the pairs [qa, qb) (slab q - qa of X, precision R);
// block row blockIdx.y takes an equal share of them.
template <int LA, class R>
__global__ FFT_BOUNDS_R(R, LA) void k_ndct_passA(Geo g, int qa, int qb, int QG, const double* __restrict__ chat,
                                        int64_t chat_stride, cplxT<R>* __restrict__ X, int64_t x_stride) {
    __shared__ cplxT<R> buf[TILE_LDS(LA)];
    STAGE_TW(stw, LA, R);
    const cplxT<R>* twA = stage_twiddles<LA, R>(stw, g.twN2, g.N2);
    const Tile<LA> T(g.colsA, g.N2);
    const int N = g.N;
    const int na0 = xcd_tile(blockIdx.x, gridDim.x) * T.cols();
    const int grp = blockIdx.y;
    const int b = blockIdx.z;
    const double* cb = chat + b * chat_stride;
    cplxT<R>* Xb = X + b * x_stride;
    const PassAOut<LA, false> out(g, T, na0);
    HeldPut<LA, false, R> held(out, g, T);
    const double invN = 1.0 / N;
    // W = A x^{2q} + B y^{2q} with A = e (1+x) chat_n / 2, B = -i e x chat_{N-n} / 2;
    // Ap = A x^{2q} and Bp = B y^{2q} are carried from pair to pair
    cplx Ap[FFT_VPT], Bp[FFT_VPT];
    const int q0 = qa + ((qb - qa) * grp) / QG, q1 = qa + ((qb - qa) * (grp + 1)) / QG;
    cplx eh[FFT_VPT];  // e^{i pi n/(2N)} of the thread's elements
    if constexpr (LA > 0) half_shift_eighths(g, na0 + T.col(0) + g.N1 * T.idx(0), eh);
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        Ap[s] = Bp[s] = {0, 0};
        if (T.live(s)) {
            const int n = na0 + T.col(s) + g.N1 * T.idx(s);
            if (n == 0) {
                if (q0 == 0) Ap[s] = {cb[0], 0};
            } else {
                const double x = n * invN, y = (N - n) * invN;
                const cplx e2 = cscale((LA > 0) ? eh[s] : half_shift_tab(g, n), 0.5);
                double a = 1, bb = 1;
                for (int q = 0; q < q0; ++q) {
                    a *= x * x;
                    bb *= y * y;
                }
                Ap[s] = cscale(e2, (1.0 + x) * cb[n] * a);
                Bp[s] = cscale(cmuli(e2), -x * cb[N - n] * bb);
            }
        }
    }
    if constexpr (sizeof(R) < sizeof(double)) {
        // FP32 terms: the carried products and the squares in FP32 (their
        // rounding is that of the FP32 terms themselves)
        cplxT<R> Af[FFT_VPT], Bf[FFT_VPT];
        R xx[FFT_VPT], yy[FFT_VPT];
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            const int n = na0 + T.col(s) + g.N1 * T.idx(s);
            const double x = n * invN, y = (N - n) * invN;
            Af[s] = cto<R>(Ap[s]);
            Bf[s] = cto<R>(Bp[s]);
            xx[s] = (R)((n == 0) ? 0.0 : x * x);
            yy[s] = (R)(y * y);
        }
        for (int q = q0; q < q1; ++q) {
            cplxT<R> v[FFT_VPT];
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) {
                v[s] = cadd(Af[s], Bf[s]);
                Af[s] = cscale(Af[s], xx[s]);
                Bf[s] = cscale(Bf[s], yy[s]);
            }
            tile_fft<LA>(v, buf, twA, T, held);
            held.hold(v, Xb + (int64_t)(q - qa) * N);
        }
    } else {
        for (int q = q0; q < q1; ++q) {
            cplxT<R> v[FFT_VPT];
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) {
                const int n = na0 + T.col(s) + g.N1 * T.idx(s);
                const double x = n * invN, y = (N - n) * invN;
                v[s] = cto<R>(cadd(Ap[s], Bp[s]));
                Ap[s] = cscale(Ap[s], (n == 0) ? 0.0 : x * x);
                Bp[s] = cscale(Bp[s], y * y);
            }
            tile_fft<LA>(v, buf, twA, T, held);
            held.hold(v, Xb + (int64_t)(q - qa) * N);
        }
    }
    held.flush();
}

// One Taylor pair per block, in FP64: pair q = qa + blockIdx.y into slab
// blockIdx.y of X.  Used where every group of the pairs holds one pair (small
// transforms, and the FP64 first pair of the FP32-bulk mode, whose other pairs
// go through k_ndct_passA<LA, float>): the input of pass A for pair q, one
// transform, the stores at once.  Without the carried powers and the held
// stores of the multi-pair pass its registers fit three or four waves per
// SIMD.  Same values as k_ndct_passA<LA, double> with one pair per group.
template <int LA>
__global__ __launch_bounds__(FFT_THREADS) __attribute__((amdgpu_waves_per_eu(LA > 0 ? 3 : FFT_WAVES)))
void k_ndct_pair(Geo g, int qa, const double* __restrict__ chat, int64_t chat_stride, cplx* __restrict__ X,
                 int64_t x_stride) {
    __shared__ cplx buf[TILE_LDS(LA)];
    STAGE_TW(stw, LA, double);
    const cplx* twA = stage_twiddles<LA, double>(stw, g.twN2, g.N2);
    const Tile<LA> T(g.colsA, g.N2);
    const int N = g.N;
    const int na0 = xcd_tile(blockIdx.x, gridDim.x) * T.cols();
    const int q = qa + (int)blockIdx.y;
    const int b = blockIdx.z;
    const double* cb = chat + b * chat_stride;
    const PassAOut<LA, false> out(g, T, na0);
    const double invN = 1.0 / N;
    cplx eh[FFT_VPT];  // e^{i pi n/(2N)} of the thread's elements
    if constexpr (LA > 0) half_shift_eighths(g, na0 + T.col(0) + g.N1 * T.idx(0), eh);
    cplx v[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        v[s] = {0, 0};
        if (T.live(s)) {
            const int n = na0 + T.col(s) + g.N1 * T.idx(s);
            if (n == 0) {
                if (q == 0) v[s] = {cb[0], 0};
            } else {
                const double x = n * invN, y = (N - n) * invN;
                double a = 1, bb = 1;  // x^{2q}, y^{2q}
                for (int k = 0; k < q; ++k) {
                    a *= x * x;
                    bb *= y * y;
                }
                const cplx e2 = cscale((LA > 0) ? eh[s] : half_shift_tab(g, n), 0.5);
                v[s] = cadd(cscale(e2, (1.0 + x) * cb[n] * a), cscale(cmuli(e2), -x * cb[N - n] * bb));
            }
        }
    }
    tile_fft<LA>(v, buf, twA, T);
    out.put(g, v, X + b * x_stride + (int64_t)blockIdx.y * N, T);
}

// Largest |d_k| = |N dtheta_k| the Taylor lengths are chosen for (pi/2, with
// room for rounding): outputs at points beyond it are NaN instead of values
// with an error above the stated bound (caller-given offsets of
// cheb_eval_nodes; the Legendre nodes and the ragged pairing stay within it).
constexpr double TAYLOR_D_MAX = 1.5707963267948966 * (1.0 + 1e-12);

// f_k = sum_l s_l d_k^l/l! F_l[k], s_l = (-1)^floor((l+1)/2), d_k = N dtheta_k,
// by Horner from the highest pair down, in FP64.  Pairs q >= 1 come from X1
// (slab q - 1, precision R), pair 0 from X0 (FP64); the next pair's tile is
// loaded while the current one is transformed.
template <int LB, class R>
__global__ FFT_BOUNDS_R(R, LB) void k_ndct_passB(Geo g, int Q, const cplx* __restrict__ X0, int64_t x0_stride,
                                        const cplxT<R>* __restrict__ X1, int64_t x1_stride,
                                        const double* __restrict__ dth, double* __restrict__ f, int64_t f_stride,
                                        RaggedRows RR) {
    __shared__ cplx bufd[TILE_LDS(LB)];
    cplxT<R>* bufr = reinterpret_cast<cplxT<R>*>(bufd);
    STAGE_TW(stwd, LB, double);
    const cplx* twd = stage_twiddles<LB, double>(stwd, g.twN1, g.N1);
    const cplxT<R>* twr;
    if constexpr (sizeof(R) == sizeof(double)) {
        twr = (const cplxT<R>*)twd;
    } else {
        STAGE_TW(stwr, LB, R);
        twr = stage_twiddles<LB, R>(stwr, g.twN1, g.N1);
    }
    const Tile<LB> T(g.rowsB, g.N1);
    const int N = g.N;
    const int jb0 = xcd_tile_mirror(blockIdx.x, gridDim.x) * T.cols();
    const int b = blockIdx.z;
    const cplx* X0b = X0 + b * x0_stride;
    const cplxT<R>* X1b = X1 + b * x1_stride;
    if constexpr (sizeof(R) < sizeof(double) && LB > 0) {
        // Pairs Q-1..1 in R from two prefetch buffers taken in turn (nxr
        // holds pairs Q-1, Q-3, ..., nyr pairs Q-2, Q-4, ...); their Horner
        // steps run in R into a partial sum accr, widened once before pair 0
        // (its rounding, relative to a partial sum that pair 0 weights by at
        // most 0.84^2/2, is that of the R terms themselves).  Pair 0 (FP64)
        // and its node offsets in FP64 are read only after the loop, so the
        // loop's registers fit three waves per SIMD.
        cplxT<R> nxr[FFT_VPT] = {}, nyr[FFT_VPT] = {};
        if (Q > 1) passB_load<LB, R>(g, jb0, X1b + (int64_t)(Q - 2) * N, nxr, T);
        if (Q > 2) passB_load<LB, R>(g, jb0, X1b + (int64_t)(Q - 3) * N, nyr, T);
        R accr[FFT_VPT], dr[FFT_VPT], sg[FFT_VPT];
        int kn[FFT_VPT];  // output index: grid row, or the node paired with it (-1: none)
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            const int m = jb0 + T.col(s) + g.N2 * T.idx(s);
            const int r = row_of(m, N);
            double dd;
            if (RR.gk) {
                kn[s] = RR.gk[(int64_t)b * N + r];
                dd = (kn[s] >= 0) ? RR.dg[(int64_t)b * N + r] : 0.0;
            } else {
                kn[s] = r;
                dd = (double)N * dth[r];
            }
            accr[s] = 0;
            dr[s] = (R)dd;
            sg[s] = (2 * m >= N) ? (R)-1 : (R)1;
        }
        auto horner_r = [&](int q, const cplxT<R>* U) {
            const R sc = (q & 1) ? (R)-1 : (R)1;
            const R r1 = (R)1 / (R)(2 * q + 1), r2 = (R)1 / (R)(2 * q + 2);
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) {
                const R inner = fmaf(dr[s] * r2, accr[s], -sc * sg[s] * U[s].im);
                accr[s] = fmaf(dr[s] * r1, inner, sc * U[s].re);
            }
        };
        for (int q = Q - 1; q >= 1; q -= 2) {
            cplxT<R> z[FFT_VPT];
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) z[s] = nxr[s];
            if (q > 2) passB_load<LB, R>(g, jb0, X1b + (int64_t)(q - 3) * N, nxr, T);
            tile_fft<LB>(z, bufr, twr, T);
            horner_r(q, z);
            if (q == 1) break;
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) z[s] = nyr[s];
            if (q > 3) passB_load<LB, R>(g, jb0, X1b + (int64_t)(q - 4) * N, nyr, T);
            tile_fft<LB>(z, bufr, twr, T);
            horner_r(q - 1, z);
        }
        // pair 0 in FP64
        cplx z0[FFT_VPT];
        passB_load<LB, double>(g, jb0, X0b, z0, T);
        double acc[FFT_VPT], d[FFT_VPT];
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            const int m = jb0 + T.col(s) + g.N2 * T.idx(s);
            const int r = row_of(m, N);
            acc[s] = (double)accr[s];
            if (RR.gk) d[s] = (kn[s] >= 0) ? RR.dg[(int64_t)b * N + r] : 0.0;
            else d[s] = (double)N * dth[r];
        }
        tile_fft<LB>(z0, bufd, twd, T);
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            const int m = jb0 + T.col(s) + g.N2 * T.idx(s);
            const double Fs = (2 * m >= N) ? -z0[s].im : z0[s].im;
            const double inner = fma(d[s] * 0.5, acc[s], -Fs);
            acc[s] = fma(d[s], inner, z0[s].re);
        }
        double* fb = RR.gk ? f + RR.offs[b] : f + b * f_stride;
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s)
            if (kn[s] >= 0) fb[kn[s]] = (fabs(d[s]) <= TAYLOR_D_MAX) ? acc[s] : __builtin_nan("");
        return;
    }
    double acc[FFT_VPT], d[FFT_VPT];
    int kn[FFT_VPT];  // output index: grid row, or the node paired with it (-1: none)
    // the first tile's loads go out before the node offsets' (loads retire
    // in order: waiting for the tile then does not wait for them)
    cplx nx[FFT_VPT] = {};
    cplxT<R> nxr[FFT_VPT] = {};
    if constexpr (sizeof(R) == sizeof(double)) {
        passB_load<LB, double>(g, jb0, X0b + (int64_t)(Q - 1) * N, nx, T);
    } else {
        if (Q > 1) passB_load<LB, R>(g, jb0, X1b + (int64_t)(Q - 2) * N, nxr, T);
        else passB_load<LB, double>(g, jb0, X0b, nx, T);
    }
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        acc[s] = 0;
        d[s] = 0;
        kn[s] = -1;
        if (T.live(s)) {
            const int m = jb0 + T.col(s) + g.N2 * T.idx(s);
            const int r = row_of(m, N);
            if (RR.gk) {
                kn[s] = RR.gk[(int64_t)b * N + r];
                d[s] = (kn[s] >= 0) ? RR.dg[(int64_t)b * N + r] : 0.0;
            } else {
                kn[s] = r;
                d[s] = (double)N * dth[r];
            }
        }
    }
    auto horner = [&](int q, const cplx* U) {
        const double sc = (q & 1) ? -1.0 : 1.0;  // s_{2q} = (-1)^q, s_{2q+1} = -(-1)^q
        const double r1 = 1.0 / (2 * q + 1), r2 = 1.0 / (2 * q + 2);
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            const int m = jb0 + T.col(s) + g.N2 * T.idx(s);
            const double Fs = (2 * m >= N) ? -U[s].im : U[s].im;
            const double inner = fma(d[s] * r2, acc[s], -sc * Fs);
            acc[s] = fma(d[s] * r1, inner, sc * U[s].re);
        }
    };
    if constexpr (sizeof(R) == sizeof(double)) {
        // all pairs FP64 and contiguous (X1 = X0 + N): two prefetch buffers
        // taken in turn, so two tiles are in flight while one is transformed
        // (nx holds pair q, ny pair q - 1)
        cplx ny[FFT_VPT] = {};
        if (Q > 1) passB_load<LB, double>(g, jb0, X0b + (int64_t)(Q - 2) * N, ny, T);
        for (int q = Q - 1; q >= 0; q -= 2) {
            cplx z[FFT_VPT];
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) z[s] = nx[s];
            if (q > 1) passB_load<LB, double>(g, jb0, X0b + (int64_t)(q - 2) * N, nx, T);
            tile_fft<LB>(z, bufd, twd, T);
            horner(q, z);
            if (q == 0) break;
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) z[s] = ny[s];
            if (q > 2) passB_load<LB, double>(g, jb0, X0b + (int64_t)(q - 3) * N, ny, T);
            tile_fft<LB>(z, bufd, twd, T);
            horner(q - 1, z);
        }
    } else {
        // pairs Q-1..1 in precision R (run-time length: one prefetch buffer,
        // nxr), pair 0 FP64 (nx)
        for (int q = Q - 1; q >= 1; --q) {
            cplxT<R> z[FFT_VPT];
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) z[s] = nxr[s];
            if (q > 1) passB_load<LB, R>(g, jb0, X1b + (int64_t)(q - 2) * N, nxr, T);
            else passB_load<LB, double>(g, jb0, X0b, nx, T);
            tile_fft<LB>(z, bufr, twr, T);
            cplx U[FFT_VPT];
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) U[s] = cwide(z[s]);
            horner(q, U);
        }
        tile_fft<LB>(nx, bufd, twd, T);
        horner(0, nx);
    }
    double* fb = RR.gk ? f + RR.offs[b] : f + b * f_stride;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s)
        if (kn[s] >= 0) fb[kn[s]] = (fabs(d[s]) <= TAYLOR_D_MAX) ? acc[s] : __builtin_nan("");
}


// ===================================================== theta^cheb* grid ===
// f_k = sum_n chat_n cos(n theta_k) with theta_k = theta*_k + delta_k,
// theta*_k = (k+3/4) alpha, alpha = 2 pi/(2N+1) (Sec. 2.2), by the Taylor
// series of Sec. 2.3 about theta*_k:
//   f_k = Re sum_l (d_k^l/l!) i^l E_l(k),  d_k = N delta_k,
//   E_l(k) = sum_{n<N} (n/N)^l chat_n e^{i n theta*_k}.
// Each E_l is a chirp-z transform, e^{i alpha k^2/2} (u_l * h)(k) with
// u_l[n] = (n/N)^l chat_n e^{i alpha (n^2/2 + 3n/4)} and h[m] = e^{-i alpha m^2/2},
// a cyclic convolution of length M = 2N computed as F^-(F^+ u_l . F^+ h)/M.
// Three passes over L slabs of M values: pass A of F^+ u_l (k_star_passA),
// pass B of F^+, the product with H = F^+ h/M and pass B of the conjugate
// transform in place (k_star_passB), pass A of the conjugate transform with
// the Horner sum over l and the output chirp (k_star_passC).  Between the
// passes the data keep the blocked layout of the other transforms.
// The transposed evaluation of the inverse transform (Sec. 4),
//   y_n = sum_k g_k cos(n theta_k) = Re sum_l (n/N)^l i^l G_l(n),
//   G_l(n) = sum_{k<N} (g_k d_k^l/l!) e^{i n theta*_k},
// is the same convolution with the chirps' roles exchanged: the input
// chirp e^{i alpha k^2/2} on g_k d_k^l/l!, the output chirp
// e^{i alpha (n^2/2 + 3n/4)}, and the Horner sum in n/N.

// e^{i pi r/den} for 0 <= r < 2 den (r an exact integer reduction)
__device__ __forceinline__ cplx cispi_frac(int64_t r, int64_t den) {
    double sn, cs;
    sincospi((double)r / (double)den, &sn, &cs);
    return {cs, sn};
}
// the input chirp e^{i alpha (n^2/2 + 3n/4)} = e^{i pi (2n^2 + 3n)/(2P)}, P = 2N+1
__device__ __forceinline__ cplx star_chirp_in(int64_t n, int64_t P) {
    return cispi_frac((2 * n * n + 3 * n) % (4 * P), 2 * P);
}
// the output chirp e^{i alpha k^2/2} = e^{i pi k^2/P}
__device__ __forceinline__ cplx star_chirp_out(int64_t k, int64_t P) {
    return cispi_frac((k * k) % (2 * P), P);
}

// Pass A of F^+ over M = 2N for the terms [qa, qb) (slab l - qa of X; block
// row blockIdx.y takes an equal share of them), inputs zero for n >= N.
// mode 0: the terms (n/N)^l chat_n of the evaluation (`in` = chat);
// mode 2: the terms g_k d_k^l/l! of the transposed evaluation, g = wts * in
// (`in` = f), d_k from the node offsets dth;
// mode 1: the cyclic chirp h~[j] = h[j] (j < N), h[2N - j] (j > N), 0
// (j = N), into slab 0.
template <int LA>
__global__ FFT_BOUNDS void k_star_passA(Geo g, int N, int qa, int qb, int QG, int mode,
                                        const double* __restrict__ chat, int64_t chat_stride,
                                        const double* __restrict__ wts, const double* __restrict__ dth,
                                        cplx* __restrict__ X, int64_t x_stride) {
    __shared__ cplx buf[TILE_LDS(LA)];
    STAGE_TW(stw, LA, double);
    const cplx* twA = stage_twiddles<LA, double>(stw, g.twN2, g.N2);
    const Tile<LA> T(g.colsA, g.N2);
    const int M = g.N;
    const int64_t P = 2 * (int64_t)N + 1;
    const int na0 = xcd_tile(blockIdx.x, gridDim.x) * T.cols();
    const int b = blockIdx.z;
    const double* cb = chat + b * chat_stride;
    cplx* Xb = X + b * x_stride;
    const PassAOut<LA, false> out(g, T, na0);
    HeldPut<LA, false, double> held(out, g, T);
    if (mode == 1) {
        cplx v[FFT_VPT];
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            v[s] = {0, 0};
            const int j = na0 + T.col(s) + g.N1 * T.idx(s);
            if (T.live(s) && j != N) v[s] = cconj(star_chirp_out(j < N ? j : M - j, P));
        }
        tile_fft<LA>(v, buf, twA, T, held);
        held.hold(v, Xb);
        held.flush();
        return;
    }
    const double invN = 1.0 / N;
    const double dsh = M_PI / (2.0 * (double)P);
    const int q0 = qa + ((qb - qa) * (int)blockIdx.y) / QG, q1 = qa + ((qb - qa) * ((int)blockIdx.y + 1)) / QG;
    // A: the term-l input times the input chirp, carried from term to term
    // by the factor r: (n/N)^l chat_n e^{i alpha (n^2/2 + 3n/4)}, r = n/N
    // (mode 0); g_k d_k^l/l! e^{i alpha k^2/2}, r = d_k/(l+1) (mode 2)
    cplx A[FFT_VPT];
    double r[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        A[s] = {0, 0};
        r[s] = 0;
        const int n = na0 + T.col(s) + g.N1 * T.idx(s);
        if (T.live(s) && n < N) {
            if (mode == 0) {
                r[s] = n * invN;
                double a = cb[n];
                for (int l = 0; l < q0; ++l) a *= r[s];
                A[s] = cscale(star_chirp_in(n, P), a);
            } else {
                r[s] = (double)N * dth[n] + dsh * (double)(2 * n - N + 1);
                double a = wts[n] * cb[n];
                for (int l = 0; l < q0; ++l) a *= r[s] / (l + 1);
                A[s] = cscale(star_chirp_out(n, P), a);
            }
        }
    }
    for (int l = q0; l < q1; ++l) {
        cplx v[FFT_VPT];
        const double fl = (mode == 0) ? 1.0 : 1.0 / (l + 1);
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            v[s] = A[s];
            A[s] = cscale(A[s], r[s] * fl);
        }
        tile_fft<LA>(v, buf, twA, T, held);
        held.hold(v, Xb + (int64_t)(l - qa) * M);
    }
    held.flush();
}

// Pass B of F^+ over the nterm slabs of X in place; then, unless fwd_only,
// the product with H and pass B of the conjugate transform: the slab holds
// Y = F+_B(conj(F+_B(x) H)), the conjugate of the inverse pass B output.
// With fwd_only the transform is scaled by 1/M instead (forming H).
template <int LB>
__global__ FFT_BOUNDS void k_star_passB(Geo g, int nterm, int fwd_only, const cplx* __restrict__ H,
                                        cplx* __restrict__ X, int64_t x_stride) {
    __shared__ cplx buf[TILE_LDS(LB)];
    STAGE_TW(stw, LB, double);
    const cplx* tw = stage_twiddles<LB, double>(stw, g.twN1, g.N1);
    const Tile<LB> T(g.rowsB, g.N1);
    const int M = g.N;
    const int vb0 = xcd_tile(blockIdx.x, gridDim.x) * T.cols();
    const int64_t off = (int64_t)(vb0 >> g.lrB) * ((int64_t)g.N1 << g.lrB);
    cplx* Xb = X + blockIdx.z * x_stride + off;
    cplx h[FFT_VPT];
    if (!fwd_only) passB_load<LB, double>(g, vb0, H, h, T);
    const double invM = 1.0 / M;
    cplx nx[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s)
        if (T.live(s)) nx[s] = Xb[threadIdx.x + s * FFT_THREADS];
    for (int t = 0; t < nterm; ++t) {
        cplx v[FFT_VPT];
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) v[s] = nx[s];
        if (t + 1 < nterm) {  // the next slab's tile loads while this one is transformed
            const cplx* src = Xb + (int64_t)(t + 1) * M;
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s)
                if (T.live(s)) nx[s] = src[threadIdx.x + s * FFT_THREADS];
        }
        tile_fft<LB>(v, buf, tw, T);
        if (fwd_only) {
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) v[s] = cscale(v[s], invM);
        } else {
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) v[s] = cconj(cmul(v[s], h[s]));
            tile_fft<LB>(v, buf, tw, T);
        }
        cplx* dst = Xb + (int64_t)t * M;
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s)
            if (T.live(s)) dst[threadIdx.x + s * FFT_THREADS] = v[s];
    }
}

// Pass A of the conjugate transform for the L slabs (term l in slab l), from
// the highest term down, with the Horner sum
//   S = a_{L-1};  S = a_l + (d_k/(l+1)) S,  a_l = i^l conj(F+_A(Y_l twiddled)),
// then f_k = Re(e^{i alpha k^2/2} S) for the outputs k < N;
// d_k = N (theta_k - theta*_k) = N dth_k + pi (2k - N + 1)/(2(2N+1)), dth
// the node offsets from theta^cheb1.  With trans (the transposed
// evaluation): S = a_l + (n/N) S and y_n = Re(e^{i alpha (n^2/2 + 3n/4)} S).
template <int LA>
__global__ FFT_BOUNDS void k_star_passC(Geo g, int N, int L, int trans, const cplx* __restrict__ X, int64_t x_stride,
                                        const double* __restrict__ dth, double* __restrict__ f, int64_t f_stride) {
    __shared__ cplx buf[TILE_LDS(LA)];
    STAGE_TW(stw, LA, double);
    const cplx* twA = stage_twiddles<LA, double>(stw, g.twN2, g.N2);
    const Tile<LA> T(g.colsA, g.N2);
    const int M = g.N;
    const int64_t P = 2 * (int64_t)N + 1;
    const int na0 = xcd_tile(blockIdx.x, gridDim.x) * T.cols();
    const int b = blockIdx.z;
    const cplx* Xb = X + b * x_stride;
    const PassAOut<LA, false> tw(g, T, na0);
    int off[FFT_VPT];
    double d[FFT_VPT];
    bool out[FFT_VPT];
    const double dsh = M_PI / (2.0 * (double)P);
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        const int na = na0 + T.col(s), k = na + g.N1 * T.idx(s);
        off[s] = passA_offset(g, na, T.idx(s), false);
        out[s] = T.live(s) && k < N;
        d[s] = !out[s] ? 0.0 : trans ? (double)k / N : (double)N * dth[k] + dsh * (double)(2 * k - N + 1);
    }
    cplx S[FFT_VPT], nx[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        S[s] = {0, 0};
        nx[s] = T.live(s) ? Xb[(int64_t)(L - 1) * M + off[s]] : cplx{0, 0};
    }
    for (int l = L - 1; l >= 0; --l) {
        cplx v[FFT_VPT];
        tw.twid(nx, v);
        if (l > 0) {
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s)
                if (T.live(s)) nx[s] = Xb[(int64_t)(l - 1) * M + off[s]];
        }
        tile_fft<LA>(v, buf, twA, T);
        const double r = trans ? 1.0 : 1.0 / (l + 1);
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            const cplx z = cconj(v[s]);
            cplx a;  // i^l z
            switch (l & 3) {
                case 0: a = z; break;
                case 1: a = {-z.im, z.re}; break;
                case 2: a = {-z.re, -z.im}; break;
                default: a = {z.im, -z.re}; break;
            }
            const double c = d[s] * r;
            S[s] = {fma(c, S[s].re, a.re), fma(c, S[s].im, a.im)};
        }
    }
    double* fb = f + b * f_stride;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        if (out[s]) {
            const int k = na0 + T.col(s) + g.N1 * T.idx(s);
            const cplx c2 = trans ? star_chirp_in(k, P) : star_chirp_out(k, P);
            fb[k] = c2.re * S[s].re - c2.im * S[s].im;
        }
    }
}

// ============================================================== inverse ===
// c = D_s M^T T^T D_w f (Sec. 4): g = w f; y = T^T g by the transposed Taylor
// series; c_n = (n+1/2) (M^T y)_n with M^T = P^T C D_eps on the grid.

// Transposed Taylor pair q: DFT input at m (row k = j(m)):
//   g_k d_k^{2q} (1 + i sigma_m d_k),  sigma_m = +1 (2m < N), -1 otherwise.
// One launch covers the pairs [qa, qb) (slab q - qa of X, precision R);
// block row blockIdx.y takes an equal share of them.
template <int LA, class R>
__global__ FFT_BOUNDS_R(R, LA) void k_tndct_passA(Geo g, int qa, int qb, int QG, const double* __restrict__ fv,
                                         int64_t f_stride, const double* __restrict__ wts,
                                         const double* __restrict__ dth, cplxT<R>* __restrict__ X, int64_t x_stride,
                                         RaggedRows RR) {
    __shared__ cplxT<R> buf[TILE_LDS(LA)];
    STAGE_TW(stw, LA, R);
    const cplxT<R>* twA = stage_twiddles<LA, R>(stw, g.twN2, g.N2);
    const Tile<LA> T(g.colsA, g.N2);
    const int N = g.N;
    const int na0 = xcd_tile_mirror(blockIdx.x, gridDim.x) * T.cols();
    const int grp = blockIdx.y;
    const int b = blockIdx.z;
    const double* fb = fv + b * f_stride;
    cplxT<R>* Xb = X + b * x_stride;
    const PassAOut<LA, true> out(g, T, na0);
    HeldPut<LA, true, R> held(out, g, T);
    double gv[FFT_VPT], dv[FFT_VPT], d2[FFT_VPT];
    const int q0 = qa + ((qb - qa) * grp) / QG, q1 = qa + ((qb - qa) * (grp + 1)) / QG;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        gv[s] = dv[s] = d2[s] = 0;
        if (T.live(s)) {
            const int m = na0 + T.col(s) + g.N1 * T.idx(s);
            const int r = row_of(m, N);
            double d, p;
            if (RR.gk) {
                const int kk = RR.gk[(int64_t)b * N + r];
                d = (kk >= 0) ? RR.dg[(int64_t)b * N + r] : 0.0;
                p = (kk >= 0) ? RR.wg[(int64_t)b * N + r] * fv[RR.offs[b] + kk] : 0.0;
            } else {
                d = (double)N * dth[r];
                p = wts[r] * fb[r];
            }
            for (int q = 0; q < q0; ++q) p *= d * d;
            gv[s] = p;  // g_k d_k^{2q}
            d2[s] = d * d;
            dv[s] = (2 * m < N) ? d : -d;  // sigma_m d_k
        }
    }
    for (int q = q0; q < q1; ++q) {
        cplxT<R> v[FFT_VPT];
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            v[s] = cto<R>(cplx{gv[s], gv[s] * dv[s]});
            gv[s] *= d2[s];
        }
        tile_fft<LA>(v, buf, twA, T, held);
        held.hold(v, Xb + (int64_t)(q - qa) * N);
    }
    held.flush();
}

// One transposed Taylor pair per block, in FP64 (as k_ndct_pair for the
// forward evaluation): pair q = qa + blockIdx.y into slab blockIdx.y of X.
// Same values as k_tndct_passA<LA, double> with one pair per group.
template <int LA>
__global__ __launch_bounds__(FFT_THREADS) __attribute__((amdgpu_waves_per_eu(LA > 0 ? 3 : FFT_WAVES)))
void k_tndct_pair(Geo g, int qa, const double* __restrict__ fv, int64_t f_stride, const double* __restrict__ wts,
                  const double* __restrict__ dth, cplx* __restrict__ X, int64_t x_stride, RaggedRows RR) {
    __shared__ cplx buf[TILE_LDS(LA)];
    STAGE_TW(stw, LA, double);
    const cplx* twA = stage_twiddles<LA, double>(stw, g.twN2, g.N2);
    const Tile<LA> T(g.colsA, g.N2);
    const int N = g.N;
    const int na0 = xcd_tile_mirror(blockIdx.x, gridDim.x) * T.cols();
    const int q = qa + (int)blockIdx.y;
    const int b = blockIdx.z;
    const double* fb = fv + b * f_stride;
    const PassAOut<LA, true> out(g, T, na0);
    cplx v[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        v[s] = {0, 0};
        if (T.live(s)) {
            const int m = na0 + T.col(s) + g.N1 * T.idx(s);
            const int r = row_of(m, N);
            double d, p;
            if (RR.gk) {
                const int kk = RR.gk[(int64_t)b * N + r];
                d = (kk >= 0) ? RR.dg[(int64_t)b * N + r] : 0.0;
                p = (kk >= 0) ? RR.wg[(int64_t)b * N + r] * fv[RR.offs[b] + kk] : 0.0;
            } else {
                d = (double)N * dth[r];
                p = wts[r] * fb[r];
            }
            for (int k = 0; k < q; ++k) p *= d * d;     // g_k d_k^{2q}
            v[s] = cplx{p, p * ((2 * m < N) ? d : -d)};  // and times sigma_m d_k
        }
    }
    tile_fft<LA>(v, buf, twA, T);
    out.put(g, v, X + b * x_stride + (int64_t)blockIdx.y * N, T);
}

// y_n = sum_l s_l (n/N)^l / l! Z_l[n]; Z_{2q} = Re(e_n A_n), Z_{2q+1} = Im(e_n B_n),
// A = (U_n + conj U_{N-n})/2, B = (U_n - conj U_{N-n})/(2i), e_n = e^{i pi n/(2N)}.
// U_{N-n} of (virtual) row i, column j_a sits in the same tile: row 0 pairs
// with itself at (N1 - j_a) mod N1, row N2/2 with itself at N1-1-j_a, row r
// with its neighbour N2 - r (virtual row i ^ 1) at N1-1-j_a; the transform
// goes through LDS once more to reach it.  Pairs q >= 1 come from X1 (slab
// q - 1, precision R), pair 0 from X0 (FP64); Horner in FP64.
template <int LB, class R>
__global__ FFT_BOUNDS void k_tndct_passB(Geo g, int Q, const cplx* __restrict__ X0, int64_t x0_stride,
                                         const cplxT<R>* __restrict__ X1, int64_t x1_stride, double* __restrict__ y,
                                         int64_t y_stride) {
    __shared__ cplx bufd[TILE_LDS(LB)];
    cplxT<R>* bufr = reinterpret_cast<cplxT<R>*>(bufd);
    STAGE_TW(stwd, LB, double);
    const cplx* twd = stage_twiddles<LB, double>(stwd, g.twN1, g.N1);
    const cplxT<R>* twr;
    if constexpr (sizeof(R) == sizeof(double)) {
        twr = (const cplxT<R>*)twd;
    } else {
        STAGE_TW(stwr, LB, R);
        twr = stage_twiddles<LB, R>(stwr, g.twN1, g.N1);
    }
    const Tile<LB> T(g.rowsB, g.N1);
    const int N = g.N;
    const int N1 = T.len();
    const int N2 = g.N2;
    const int vb0 = xcd_tile(blockIdx.x, gridDim.x) * T.cols();
    const int b = blockIdx.z;
    const cplx* X0b = X0 + b * x0_stride;
    const cplxT<R>* X1b = X1 + b * x1_stride;
    double acc[FFT_VPT], xs[FFT_VPT];
    cplx en[FFT_VPT];
    int part[FFT_VPT];
    if constexpr (LB > 0) half_shift_eighths(g, actual_row(vb0 + T.col(0), N2) + N2 * T.idx(0), en);
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        acc[s] = 0;
        xs[s] = 0;
        if constexpr (LB == 0) en[s] = {0, 0};
        part[s] = 0;
        if (T.live(s)) {
            const int i = T.col(s), ja = T.idx(s);
            const int r = actual_row(vb0 + i, N2);
            const int n = r + N2 * ja;
            xs[s] = (double)n / N;
            if constexpr (LB == 0) en[s] = half_shift_tab(g, n);
            int ip, jp;
            if (r == 0) {
                ip = i;
                jp = (N1 - ja) & (N1 - 1);
            } else if (2 * r == N2) {
                ip = i;
                jp = N1 - 1 - ja;
            } else {
                ip = i ^ 1;
                jp = N1 - 1 - ja;
            }
            part[s] = Tile<LB>::sw(ip * N1 + jp);
        }
    }
    // one Horner step from each value u and its partner's value V
    auto horner = [&](int q, int s, const cplx u, const cplx V) {
        const double sc = (q & 1) ? -1.0 : 1.0;
        const double r1 = 1.0 / (2 * q + 1), r2 = 1.0 / (2 * q + 2);
        const cplx A = {0.5 * (u.re + V.re), 0.5 * (u.im - V.im)};
        const cplx Bm = {0.5 * (u.im + V.im), -0.5 * (u.re - V.re)};  // (U - conj V)/(2i)
        const double Zc = en[s].re * A.re - en[s].im * A.im;
        const double Zs = en[s].re * Bm.im + en[s].im * Bm.re;
        const double inner = fma(xs[s] * r2, acc[s], -sc * Zs);
        acc[s] = fma(xs[s] * r1, inner, sc * Zc);
    };
    // run-time length: the transformed tile in buffer `bb` (precision P)
    // goes through LDS once more to pair each value with its partner
    auto combine = [&](int q, auto* bb, const auto* U) {
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s)
            if (T.live(s)) bb[T.slot(s)] = U[s];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s)
            if (T.live(s)) horner(q, s, cwide(U[s]), cwide(bb[part[s]]));
        __syncthreads();
    };
    // compile-time length: the partner of output (col, i0 + s L/8) is output
    // (colp, i0p + sp L/8) with sp = 7 - s, or (8 - s) mod 8 for row 0 at
    // i0 = 0; the transform computes the partner thread's outputs as well
    int colp = 0, i0p = 0;
    bool z = false;
    if constexpr (LB > 0) {
        constexpr int ST = Tile<LB>::STRIDE;
        const int i = T.col_, i0 = T.i0_;
        const int r = actual_row(vb0 + i, N2);
        if (r == 0) {
            colp = i;
            i0p = (ST - i0) & (ST - 1);
            z = (i0 == 0);
        } else {
            colp = (2 * r == N2) ? i : (i ^ 1);
            i0p = ST - 1 - i0;
        }
    }
    auto transform_combine = [&](int q, auto* U, auto* bb, const auto* twb) {
        if constexpr (LB > 0) {
            using V_t = std::remove_reference_t<decltype(U[0])>;
            V_t VP[FFT_VPT];
            tile_fft_with<LB>(U, VP, bb, twb, T, colp, i0p);
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) horner(q, s, cwide(U[s]), cwide(z ? VP[(8 - s) & 7] : VP[7 - s]));
        } else {
            tile_fft<LB>(U, bb, twb, T);
            combine(q, bb, U);
        }
    };
    if constexpr (sizeof(R) == sizeof(double) && LB == 0) {
        // all pairs FP64 and contiguous (X1 = X0 + N); run-time length (short
        // transforms): one prefetch buffer, within the registers
        cplx nx[FFT_VPT] = {};
        passB_load<LB, double>(g, vb0, X0b + (int64_t)(Q - 1) * N, nx, T);
        for (int q = Q - 1; q >= 0; --q) {
            cplx U[FFT_VPT];
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) U[s] = nx[s];
            if (q > 0) passB_load<LB, double>(g, vb0, X0b + (int64_t)(q - 1) * N, nx, T);
            transform_combine(q, U, bufd, twd);
        }
    } else if constexpr (sizeof(R) == sizeof(double)) {
        // all pairs FP64 and contiguous: two prefetch buffers taken in turn
        // (nx holds pair q, ny pair q - 1)
        cplx nx[FFT_VPT] = {}, ny[FFT_VPT] = {};
        passB_load<LB, double>(g, vb0, X0b + (int64_t)(Q - 1) * N, nx, T);
        if (Q > 1) passB_load<LB, double>(g, vb0, X0b + (int64_t)(Q - 2) * N, ny, T);
        for (int q = Q - 1; q >= 0; q -= 2) {
            cplx U[FFT_VPT];
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) U[s] = nx[s];
            if (q > 1) passB_load<LB, double>(g, vb0, X0b + (int64_t)(q - 2) * N, nx, T);
            transform_combine(q, U, bufd, twd);
            if (q == 0) break;
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) U[s] = ny[s];
            if (q > 2) passB_load<LB, double>(g, vb0, X0b + (int64_t)(q - 3) * N, ny, T);
            transform_combine(q - 1, U, bufd, twd);
        }
    } else {
        cplxT<R> nx[FFT_VPT] = {};
        cplx n0[FFT_VPT] = {};
        if (Q > 1) passB_load<LB, R>(g, vb0, X1b + (int64_t)(Q - 2) * N, nx, T);
        else passB_load<LB, double>(g, vb0, X0b, n0, T);
        for (int q = Q - 1; q >= 1; --q) {
            cplxT<R> U[FFT_VPT];
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) U[s] = nx[s];
            if (q > 1) passB_load<LB, R>(g, vb0, X1b + (int64_t)(q - 2) * N, nx, T);
            else passB_load<LB, double>(g, vb0, X0b, n0, T);
            transform_combine(q, U, bufr, twr);
        }
        transform_combine(0, n0, bufd, twd);
    }
    double* yb = y + b * y_stride;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        if (T.live(s)) {
            const int r = actual_row(vb0 + T.col(s), N2);
            yb[r + N2 * T.idx(s)] = acc[s];
        }
    }
}

// (M^T y)_n for n < nd, chunk blockIdx.y of rows k:
//   sum_{k in chunk, k <= n, k+n even} (eps_k/pi) Lam((n-k)/2) Lam((n+k)/2) y_k
// Same blocking as k_dense with the roles of rows and columns exchanged.
__global__ __launch_bounds__(256) void k_dense_t(int nd, int chunk, const double* __restrict__ lam,
                                                 const double* __restrict__ y, int64_t y_stride,
                                                 double* __restrict__ part, int64_t part_stride) {
    __shared__ double sy[DENSE_CH], slm[DENSE_CH / 2 + 256], slp[DENSE_CH / 2 + 256];
    const int par = blockIdx.x & 1;
    const int nb0 = (blockIdx.x >> 1) * 512;
    const int ch = blockIdx.y;
    const int b = blockIdx.z;
    const double* yb = y + b * y_stride;
    const int k0 = ch * DENSE_CH, k1 = min(nd, k0 + DENSE_CH);
    const int n = nb0 + 2 * threadIdx.x + par;
    // (n-k)/2 in [zm0, ...): n - k >= nb0 - (k0 + CH - 1); (n+k)/2 >= (nb0 + k0)/2
    const int zm0 = (nb0 - (k0 + DENSE_CH - 1)) >> 1;
    const int zp0 = (nb0 + k0) >> 1;
#pragma unroll
    for (int i = threadIdx.x; i < DENSE_CH; i += 256) {
        int kk = k0 + i;
        sy[i] = (kk < k1) ? yb[kk] * ((kk == 0) ? 0.3183098861837907 : 0.6366197723675814) : 0.0;
    }
#pragma unroll
    for (int i = threadIdx.x; i < DENSE_CH / 2 + 256; i += 256) {
        int zm = zm0 + i, zp = zp0 + i;
        slm[i] = (zm >= 0 && zm < nd) ? lam[zm] : 0.0;
        slp[i] = (zp >= 0 && zp < nd) ? lam[zp] : 0.0;
    }
    __syncthreads();
    if (n >= nd) return;
    int kk = k0;
    if ((n - kk) & 1) ++kk;
    const int kend = min(k1, n + 1);
    // four rows per step into four sums (as in k_dense)
    int im = ((n - kk) >> 1) - zm0, ip = ((n + kk) >> 1) - zp0, iy = kk - k0;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (; kk + 6 < kend; kk += 8, im -= 4, ip += 4, iy += 8) {
        a0 = fma(slm[im] * slp[ip], sy[iy], a0);
        a1 = fma(slm[im - 1] * slp[ip + 1], sy[iy + 2], a1);
        a2 = fma(slm[im - 2] * slp[ip + 2], sy[iy + 4], a2);
        a3 = fma(slm[im - 3] * slp[ip + 3], sy[iy + 6], a3);
    }
    for (; kk < kend; kk += 2, --im, ++ip, iy += 2) a0 = fma(slm[im] * slp[ip], sy[iy], a0);
    part[b * part_stride + (int64_t)ch * nd + n] = (a0 + a1) + (a2 + a3);
}

__global__ void k_dense_t_reduce(int nd, int nchunk, int chunk, const double* __restrict__ part,
                                 int64_t part_stride, double* __restrict__ out, int64_t out_stride, int half) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.z;
    if (n >= nd) return;
    const double* pb = part + b * part_stride;
    double s = 0;
    int last = min(nchunk - 1, n / chunk);
    for (int ch = 0; ch <= last; ++ch) s += pb[(int64_t)ch * nd + n];
    out[b * out_stride + n] = half ? (n + 0.5) * s : s;
}

// u_j = sum_k (eps_k/N) y_k cos(k theta_j): DFT of (eps_k/N) y_k e^{i pi k/(2N)},
// u at row j(m) = Re V_m.
template <int LA>
__global__ FFT_BOUNDS void k_dct3_passA(Geo g, const double* __restrict__ y, int64_t y_stride,
                                                           cplx* __restrict__ X, int64_t x_stride) {
    __shared__ cplx buf[TILE_LDS(LA)];
    STAGE_TW(stw, LA, double);
    const cplx* twA = stage_twiddles<LA, double>(stw, g.twN2, g.N2);
    const Tile<LA> T(g.colsA, g.N2);
    const int N = g.N;
    const int na0 = xcd_tile(blockIdx.x, gridDim.x) * T.cols();
    const int b = blockIdx.z;
    const double* yb = y + b * y_stride;
    const PassAOut<LA, false> out(g, T, na0);
    cplx eh[FFT_VPT];  // e^{i pi n/(2N)} of the thread's elements
    if constexpr (LA > 0) half_shift_eighths(g, na0 + T.col(0) + g.N1 * T.idx(0), eh);
    cplx x[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        if (T.live(s)) {
            const int n = na0 + T.col(s) + g.N1 * T.idx(s);
            const double a = yb[n] * ((n == 0) ? 1.0 : 2.0) / N;
            x[s] = cscale((LA > 0) ? eh[s] : half_shift_tab(g, n), a);
        }
    }
    tile_fft<LA>(x, buf, twA, T);
    out.put(g, x, X + b * x_stride, T);
}

template <int LB>
__global__ FFT_BOUNDS void k_dct3_passB(Geo g, const cplx* __restrict__ X, int64_t x_stride,
                                                           double* __restrict__ u, int64_t u_stride) {
    __shared__ cplx buf[TILE_LDS(LB)];
    STAGE_TW(stw, LB, double);
    const cplx* twB = stage_twiddles<LB, double>(stw, g.twN1, g.N1);
    const Tile<LB> T(g.rowsB, g.N1);
    const int N = g.N;
    const int jb0 = xcd_tile_mirror(blockIdx.x, gridDim.x) * T.cols();
    const int b = blockIdx.z;
    cplx z[FFT_VPT];
    passB_load<LB, double>(g, jb0, X + b * x_stride, z, T);
    tile_fft<LB>(z, buf, twB, T);
    double* ub = u + b * u_stride;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        if (T.live(s)) {
            const int m = jb0 + T.col(s) + g.N2 * T.idx(s);
            ub[row_of(m, N)] = z[s].re;
        }
    }
}

// Transposed far field, pass A: for every term (b, m), ascending m, the DFT
// input at m is rho at row j = j(m) (conjugated when 2m >= N) with
//   rho_j = u_j e^{i (m+1/2)(theta_j - pi/2)} (2 sin theta_j)^{-m-1/2} [j in block b].
// Term group blockIdx.y takes the terms y, y + G, ...
template <int LA, class R>
__global__ FFT_BOUNDS_R(R, LA) void k_tfar_passA(Geo g, FarParams F, int G, const cplx* __restrict__ rowf,
                                                           const double* __restrict__ u, int64_t u_stride,
                                                           cplxT<R>* __restrict__ X, int64_t x_stride) {
    __shared__ cplxT<R> buf[TILE_LDS(LA)];
    STAGE_TW(stw, LA, R);
    const cplxT<R>* twA = stage_twiddles<LA, R>(stw, g.twN2, g.N2);
    const Tile<LA> T(g.colsA, g.N2);
    const FarTerms FT(F);
    const int N = g.N;
    const int na0 = xcd_tile_mirror(blockIdx.x, gridDim.x) * T.cols();
    const int b = blockIdx.z;
    const double* ub = u + b * u_stride;
    cplxT<R>* Xb = X + b * x_stride;
    const PassAOut<LA, false> out(g, T, na0);
    const HeldPut<LA, false, R> put(out, g, T);  // stores only (no tile held)
    cplx gm[FFT_VPT], rq[FFT_VPT];
    int key[FFT_VPT];  // 2 * block + (conjugated input), -1 outside
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        gm[s] = rq[s] = {0, 0};
        key[s] = -1;
        if (T.live(s)) {
            const int mo = na0 + T.col(s) + g.N1 * T.idx(s);
            const int j = row_of(mo, N);
            const int blk = row_block(F, j, N);
            if (blk >= 0) key[s] = 2 * blk + (2 * mo >= N ? 1 : 0);
            const cplx g0 = rowf[mo];
            rq[s] = cmul(g0, g0);
            gm[s] = cscale(g0, ub[j]);
        }
    }
    int mcur = 0;
    for (int t = blockIdx.y; t < F.nterm; t += G) {
        const int m = FT.m(t);
        const int tb = FT.blk(t);
        for (; mcur < m; ++mcur) {
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) gm[s] = cmul(gm[s], rq[s]);
        }
        cplxT<R> v[FFT_VPT];
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            v[s] = ((key[s] >> 1) == tb) ? cto<R>(gm[s]) : cplxT<R>{0, 0};
            if (key[s] & 1) v[s].im = -v[s].im;
        }
        tile_fft<LA>(v, buf, twA, T);
        put.put(v, Xb + (int64_t)t * N);
    }
}

// Transposed far field, pass B: out_n = sum_terms C_n h_{m,n} [n >= nlo_b]
// Re(e^{i pi n/(2N)} U_n), descending m (h by multiplication only); term
// group blockIdx.y takes the terms nterm-1-y, nterm-1-y-G, ... and writes
// partial sums to out[y].
template <int LB, class R>
__global__ FFT_BOUNDS void k_tfar_passB(Geo g, FarParams F, int G, const cplx* __restrict__ amp,
                                                           const cplxT<R>* __restrict__ X, int64_t x_stride,
                                                           double* __restrict__ out, int64_t out_stride) {
    __shared__ cplxT<R> buf[TILE_LDS(LB)];
    STAGE_TW(stw, LB, R);
    const cplxT<R>* twB = stage_twiddles<LB, R>(stw, g.twN1, g.N1);
    const Tile<LB> T(g.rowsB, g.N1);
    const FarTerms FT(F);
    const int N = g.N;
    const int jb0 = xcd_tile(blockIdx.x, gridDim.x) * T.cols();
    const int b = blockIdx.z;
    const cplxT<R>* Xb = X + b * x_stride;
    double acc[FFT_VPT];
    cplx eh[FFT_VPT];  // C_n h_{m,n} e^{i pi n/(2N)} at the current m
    int nn[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        acc[s] = 0;
        eh[s] = {0, 0};
        nn[s] = -1;
        if (T.live(s)) {
            const int n = jb0 + T.col(s) + g.N2 * T.idx(s);
            nn[s] = n;
            if (n >= F.nd) eh[s] = amp[n];
        }
    }
    int mcur = F.Mmax - 1;
    int t = F.nterm - 1 - (int)blockIdx.y;
    cplxT<R> nx[FFT_VPT] = {};
    if (t >= 0) passB_load<LB, R>(g, jb0, Xb + (int64_t)t * N, nx, T);
    for (; t >= 0; t -= G) {
        const int m = FT.m(t);
        const int nlo = FT.nlo(t);
        cplxT<R> U[FFT_VPT];
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) U[s] = nx[s];
        if (t - G >= 0) passB_load<LB, R>(g, jb0, Xb + (int64_t)(t - G) * N, nx, T);
        for (; mcur > m; --mcur) {
            const double fm = (double)mcur / ((mcur - 0.5) * (mcur - 0.5));
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) eh[s] = cscale(eh[s], fm * (nn[s] + mcur + 0.5));
        }
        tile_fft<LB>(U, buf, twB, T);
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s)
            if (nn[s] >= nlo) acc[s] = fma(eh[s].re, (double)U[s].re, fma(-eh[s].im, (double)U[s].im, acc[s]));
    }
    double* ob = out + b * out_stride + (int64_t)blockIdx.y * N;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s)
        if (T.live(s)) ob[nn[s]] = acc[s];
}

// Chunk-start states (once per plan): k_near_items gives each (row, chunk)
// transfer matrix and k_tnear_scan chains them per row into the state (P, D)
// at every chunk start.  Transposed near field: k_tnear_accum reruns each
// chunk from its true state for the 64 rows of one wave and sums over the rows
//   out_n += P_n(x_j) (u_j + (-1)^n u_{N-1-j})
// through an LDS tile, 32 degrees at a time; partial sums per row group.
// One wave per row: states (P, D) at every chunk start.  Lane runs of chunks
// are chained into transfer matrices, an exclusive scan over lanes gives each
// run's start state, and every lane then walks its run.
__global__ __launch_bounds__(64) void k_tnear_scan(NearParams NP, const double* __restrict__ items,
                                                   int64_t it_stride, double* __restrict__ st, int64_t st_stride) {
    const int j = blockIdx.x;
    const int b = blockIdx.z;
    const int lane = threadIdx.x;
    const int sgi = near_seg_of(NP, j);
    if (sgi < 0) return;
    const Seg S = NP.seg[sgi];
    const double* it = items + b * it_stride;
    double* so = st + b * st_stride;
    const int nrows = S.jhi - S.jlo;
    const int id0 = S.item_off + (j - S.jlo);
    const int rest = S.nchunk - 1;
    const int per = (rest + 63) / 64;
    const int c0 = 1 + lane * per, c1 = min(S.nchunk, c0 + per);
    // this lane's run as a transfer matrix [[a, c], [b, d]]
    double a = 1, bb = 0, c = 0, d = 1;
    for (int ch = c0; ch < c1; ++ch) {
        const double* q = it + (int64_t)(id0 + ch * nrows) * 8;
        double na = q[0] * a + q[2] * bb, nbv = q[1] * a + q[3] * bb;
        double nc = q[0] * c + q[2] * d, nd = q[1] * c + q[3] * d;
        a = na;
        bb = nbv;
        c = nc;
        d = nd;
    }
    // inclusive scan: T_l <- T_l T_{l-k}
    for (int k2 = 1; k2 < 64; k2 *= 2) {
        double pa = __shfl_up(a, k2), pb = __shfl_up(bb, k2), pc = __shfl_up(c, k2), pd = __shfl_up(d, k2);
        if (lane >= k2) {
            double na = a * pa + c * pb, nbv = bb * pa + d * pb;
            double nc = a * pc + c * pd, nd = bb * pc + d * pd;
            a = na;
            bb = nbv;
            c = nc;
            d = nd;
        }
    }
    // exclusive prefix = inclusive of lane-1
    double ea = __shfl_up(a, 1), eb = __shfl_up(bb, 1), ec = __shfl_up(c, 1), ed = __shfl_up(d, 1);
    if (lane == 0) {
        ea = 1;
        eb = 0;
        ec = 0;
        ed = 1;
    }
    const double* o = it + (int64_t)id0 * 8;
    double P1 = o[0], D1 = o[1];  // state after chunk 0
    double P = ea * P1 + ec * D1, D = eb * P1 + ed * D1;
    if (lane == 0) {
        so[2 * id0] = 1;
        so[2 * id0 + 1] = 0;
    }
    for (int ch = c0; ch < c1; ++ch) {
        int id = id0 + ch * nrows;
        so[2 * id] = P;
        so[2 * id + 1] = D;
        const double* q = it + (int64_t)id * 8;
        double Pn = q[0] * P + q[2] * D;
        double Dn = q[1] * P + q[3] * D;
        P = Pn;
        D = Dn;
    }
}

constexpr int TN_STEPS = 8;              // degrees per LDS tile and chain
constexpr int TN_CH = 4;                 // independent recurrences per lane
constexpr int TN_LEN = NEAR_CHUNK / TN_CH;
constexpr int TN_QUADS = TN_STEPS / 4;   // 4-degree groups per tile and chain
constexpr int TN_PITCH = 65;             // LDS pitch of one (chain, group) slot

// Lane sums of two doubles by exchanging wave halves or 16-lane rows
// (v_permlane32_swap / v_permlane16_swap, register operations):
//   sum32(x, y): lanes l < 32 get x_l + x_{l+32}, lanes l >= 32 get
//                y_{l-32} + y_l;
//   sum16(x, y): in rows R (16 lanes) 0, 1, 2, 3 the lanes get the sums of
//                lanes l, l+16 of x (row 0), of y (row 1), of x (row 2) and of
//                y (row 3), pairing rows 0/1 and 2/3.
__device__ __forceinline__ double lane_sum32(double x, double y) {
    const unsigned xl = (unsigned)__double2loint(x), xh = (unsigned)__double2hiint(x);
    const unsigned yl = (unsigned)__double2loint(y), yh = (unsigned)__double2hiint(y);
    const auto rl = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
    return __hiloint2double((int)rh[0], (int)rl[0]) + __hiloint2double((int)rh[1], (int)rl[1]);
}
__device__ __forceinline__ double lane_sum16(double x, double y) {
    const unsigned xl = (unsigned)__double2loint(x), xh = (unsigned)__double2hiint(x);
    const unsigned yl = (unsigned)__double2loint(y), yh = (unsigned)__double2hiint(y);
    const auto rl = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    return __hiloint2double((int)rh[0], (int)rl[0]) + __hiloint2double((int)rh[1], (int)rl[1]);
}

// Work-group = 64 rows of one segment and one degree chunk; each lane runs
// its row over the chunk as TN_CH recurrences of TN_LEN degrees side by side
// from the plan's states.  The products P_n(x_j) w_j of 4 consecutive degrees
// are first summed over 4 rows in registers (lane_sum32 on degree pairs, then
// lane_sum16): lane l then holds degree offset {0, 2, 1, 3}[l / 16] summed
// over rows l % 16 + {0, 16, 32, 48}.  These partials go through an LDS tile
// (a quarter of the products) where two lanes sum a degree's 16 partials;
// partial sums per row group.
__global__ __launch_bounds__(64) void k_tnear_accum(int N, NearParams NP, const int* __restrict__ wg_seg,
                                                    const int* __restrict__ segoff, const double* __restrict__ rcp,
                                                    const double* __restrict__ u, int64_t u_stride,
                                                    const double* __restrict__ st, double* __restrict__ part,
                                                    int64_t part_stride) {
    __shared__ double tile[TN_CH * TN_QUADS * TN_PITCH];
    __shared__ double sr[NEAR_CHUNK];
    const NearWG W = near_wg(NP, wg_seg, segoff, blockIdx.x);
    const Seg S = NP.seg[W.seg];
    const int n0 = W.ch * NEAR_CHUNK, n1 = min(S.nend, n0 + NEAR_CHUNK);
    if (n1 <= NP.nd) return;  // degrees below nd come from the exact low block
    const int b = blockIdx.z;
    const int nrows = S.jhi - S.jlo;
    const int row = W.grp * 64 + threadIdx.x;
    const bool act = row < nrows;
    const int j = S.jlo + (act ? row : 0);
    const int rg_global = segoff[2 * W.seg + 1] + W.grp;
    const double* ub = u + b * u_stride;
    const double uj = act ? ub[j] : 0.0, um = act ? ub[N - 1 - j] : 0.0;
    const double pi = 3.141592653589793;
    const double sn = sin(0.5 * (j + 0.5) * pi / N);
    const double uu = 2.0 * sn * sn;
    const int id = S.item_off + W.ch * nrows + (act ? row : 0);
    double p[TN_CH], d[TN_CH];
#pragma unroll
    for (int k = 0; k < TN_CH; ++k) {
        const int q = k * (NEAR_NSUB / TN_CH);
        p[k] = st[(int64_t)id * 2 * NEAR_NSUB + 2 * q];
        d[k] = st[(int64_t)id * 2 * NEAR_NSUB + 2 * q + 1];
    }
    {
        // the chunk's 1/(n+1) (rcp has N entries, a multiple of NEAR_CHUNK)
        double lr[NEAR_CHUNK / 64];
#pragma unroll
        for (int q = 0; q < NEAR_CHUNK / 64; ++q) lr[q] = rcp[n0 + (int)threadIdx.x + 64 * q];
#pragma unroll
        for (int q = 0; q < NEAR_CHUNK / 64; ++q) sr[threadIdx.x + 64 * q] = lr[q];
    }
    __syncthreads();
    double* pb = part + b * part_stride + (int64_t)rg_global * N;
    const double we = uj + um, wo = uj - um;  // weights of even / odd degrees
    // reduction: lane L sums column c = L % 32 = (chain, degree of the tile)
    // over 8 of its 16 partials, the other 8 in lane L + 32.  Lanes of rows
    // 2, 3 start half a row on, which with the odd pitch keeps each 32-lane
    // group on distinct banks.
    const int c = threadIdx.x & 31, half = threadIdx.x >> 5;
    const int kc = c / TN_STEPS, dcol = c % TN_STEPS;
    const int rsel = (dcol & 3) == 1 ? 2 : (dcol & 3) == 2 ? 1 : (dcol & 3);  // row of the degree offset
    const int rbase = (kc * TN_QUADS + (dcol >> 2)) * TN_PITCH + rsel * 16;
    const int p0 = half * 8 + (rsel >> 1) * 8;
    for (int nb = 0; nb < TN_LEN; nb += TN_STEPS) {
#pragma unroll
        for (int qd = 0; qd < TN_QUADS; ++qd) {
            double v[TN_CH][4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
#pragma unroll
                for (int k = 0; k < TN_CH; ++k) {
                    v[k][i] = p[k] * ((i & 1) ? wo : we);
                    reinsch_step(uu, sr[k * TN_LEN + nb + 4 * qd + i], p[k], d[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < TN_CH; ++k)
                tile[(k * TN_QUADS + qd) * TN_PITCH + threadIdx.x] =
                    lane_sum16(lane_sum32(v[k][0], v[k][1]), lane_sum32(v[k][2], v[k][3]));
        }
        __syncthreads();
        double s0 = 0, s1 = 0;
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
            s0 += tile[rbase + ((p0 + i) & 15)];
            s1 += tile[rbase + ((p0 + i + 1) & 15)];
        }
        const double s = lane_sum32(s0 + s1, s0 + s1);
        const int n = n0 + kc * TN_LEN + nb + dcol;
        if (half == 0 && n < n1) pb[n] = s;
        __syncthreads();
    }
}

// (M^T y)_n = dense_n [n < nd] + far_n + sum_rg near parts [nd <= n < nend(rg)],
// times n + 1/2 when `half` (the D_s of the inverse transform)
__global__ void k_idlt_final(int N, int nd, int nrg, const int* __restrict__ rg_nend, const double* __restrict__ dense,
                             int64_t dense_stride, int G, const double* __restrict__ far, int64_t far_stride,
                             const double* __restrict__ part, int64_t part_stride, double* __restrict__ c,
                             int64_t c_stride, int half) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.z;
    if (n >= N) return;
    double s;
    if (n < nd) {
        s = dense[b * dense_stride + n];
    } else {
        s = 0.0;
        for (int q = 0; q < G; ++q) s += far[b * far_stride + (int64_t)q * N + n];
        const double* pb = part + b * part_stride;
        for (int r = 0; r < nrg; ++r)
            if (n < rg_nend[r]) s += pb[(int64_t)r * N + n];
    }
    c[b * c_stride + n] = half ? (n + 0.5) * s : s;
}

}  // namespace dlt

// ================================================================ host ====
#include <hip/hip_ext.h>

// Launch a length-templated pass kernel: the compile-time length is used
// when the tile is full (N >= FFT_CAP), the run-time path otherwise.
#define LEN_LAUNCH(FULL, LEN, KER, GRID, BLK, SHM, STR, ...)                      \
    do {                                                                          \
        int L_ = (FULL) ? (LEN) : 0;                                              \
        switch (L_) {                                                             \
            case 64: launch(KER<64>, GRID, BLK, SHM, STR, __VA_ARGS__); break;         \
            case 128: launch(KER<128>, GRID, BLK, SHM, STR, __VA_ARGS__); break;       \
            case 256: launch(KER<256>, GRID, BLK, SHM, STR, __VA_ARGS__); break;       \
            case 512: launch(KER<512>, GRID, BLK, SHM, STR, __VA_ARGS__); break;       \
            case 1024: launch(KER<1024>, GRID, BLK, SHM, STR, __VA_ARGS__); break;     \
            case 2048: launch(KER<2048>, GRID, BLK, SHM, STR, __VA_ARGS__); break;     \
            default: launch(KER<0>, GRID, BLK, SHM, STR, __VA_ARGS__); break;          \
        }                                                                         \
    } while (0)
// The same for kernels with a precision parameter R (double or float).
#define LEN_LAUNCH_R(FULL, LEN, KER, R, GRID, BLK, SHM, STR, ...)                  \
    do {                                                                          \
        int L_ = (FULL) ? (LEN) : 0;                                              \
        switch (L_) {                                                             \
            case 64: launch(KER<64, R>, GRID, BLK, SHM, STR, __VA_ARGS__); break;      \
            case 128: launch(KER<128, R>, GRID, BLK, SHM, STR, __VA_ARGS__); break;    \
            case 256: launch(KER<256, R>, GRID, BLK, SHM, STR, __VA_ARGS__); break;    \
            case 512: launch(KER<512, R>, GRID, BLK, SHM, STR, __VA_ARGS__); break;    \
            case 1024: launch(KER<1024, R>, GRID, BLK, SHM, STR, __VA_ARGS__); break;  \
            case 2048: launch(KER<2048, R>, GRID, BLK, SHM, STR, __VA_ARGS__); break;  \
            default: launch(KER<0, R>, GRID, BLK, SHM, STR, __VA_ARGS__); break;       \
        }                                                                         \
    } while (0)
namespace dlt {

// ---- kernel trace: a start and an end event bound to every traced launch
namespace trace {
struct Rec {
    std::string name;
    hipEvent_t a, b;
};
static std::mutex mu;
static bool on = false;
static std::vector<Rec> recs;
static std::vector<hipEvent_t> pool;
// events of the launch being traced (null outside traced launches), and
// whether a kernel took them
static thread_local hipEvent_t cur_a = nullptr, cur_b = nullptr;
static thread_local bool used = false;

static hipEvent_t take() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}
}  // namespace trace

bool trace_on() { return trace::on; }

// Kernel launch.  Inside a traced launch the kernel takes the trace's events
// itself (hipExtLaunchKernel binds them to the dispatch), so they hold the
// kernel's own start and end, not the stream's progress before and after it.
template <class... P, class... A>
static inline void launch(void (*k)(P...), dim3 g, dim3 b, size_t shm, hipStream_t s, A&&... a) {
    if (trace::cur_a) {
        trace::used = true;
        hipExtLaunchKernelGGL(k, g, b, (std::uint32_t)shm, s, trace::cur_a, trace::cur_b, 0, static_cast<P>(a)...);
    } else {
        k<<<g, b, shm, s>>>(static_cast<P>(a)...);
    }
}

void trace_set(bool enable) {
    std::lock_guard<std::mutex> lk(trace::mu);
    trace::on = enable;
}

// current transform size, appended to trace names ("kernel/N")
static thread_local int64_t trace_n = 0;
static thread_local bool trace_held = false;
void trace_hold(bool hold) { trace_held = hold; }

// runs `fn` (one kernel launch); when tracing, the kernel records a start and
// an end event of its own

template <class F>
static void traced(const char* name, hipStream_t s, F&& fn) {
    if (!trace::on || trace_held) {
        fn();
        return;
    }
    std::lock_guard<std::mutex> lk(trace::mu);
    trace::Rec r{std::string(name) + "/" + std::to_string(trace_n), trace::take(), trace::take()};
    (void)s;  // the launch itself names its stream
    trace::cur_a = r.a;
    trace::cur_b = r.b;
    trace::used = false;
    fn();
    trace::cur_a = trace::cur_b = nullptr;
    if (trace::used) {
        trace::recs.push_back(r);
    } else {  // nothing launched
        trace::pool.push_back(r.a);
        trace::pool.push_back(r.b);
    }
}

int trace_collect(std::vector<std::pair<std::string, std::pair<double, int64_t>>>& out) {
    std::lock_guard<std::mutex> lk(trace::mu);
    std::map<std::string, std::pair<double, int64_t>> acc;
    for (auto& r : trace::recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return -3;
        float ms = 0;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return -3;
        auto& a = acc[r.name];
        a.first += ms;
        a.second += 1;
        trace::pool.push_back(r.a);
        trace::pool.push_back(r.b);
    }
    trace::recs.clear();
    out.assign(acc.begin(), acc.end());
    return 0;
}


static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

size_t work_bytes(const Plan& p, int64_t nb) { return (size_t)nb * p.ws_per_inst; }

void work_carve(const Plan& p, int64_t nb, void* base, Work& w) {
    char* q = (char*)base;
    auto take = [&](size_t per) {
        char* r = q;
        q += al256(per) * nb;
        return (void*)r;
    };
    w.X = (cplx*)take(p.ws_X);
    w.sX = (int64_t)(al256(p.ws_X) / sizeof(cplx));
    w.v = (double*)take(p.ws_v);
    w.sv = (int64_t)(al256(p.ws_v) / sizeof(double));
    w.items = (double*)take(p.ws_items);
    w.sitems = (int64_t)(al256(p.ws_items) / sizeof(double));
    w.near = (double*)take(p.ws_near);
    w.snear = (int64_t)(al256(p.ws_near) / sizeof(double));
    w.dense = (double*)take(p.ws_dense);
    w.sdense = (int64_t)(al256(p.ws_dense) / sizeof(double));
    w.chat = (double*)take(p.ws_chat);
    w.schat = (int64_t)(al256(p.ws_chat) / sizeof(double));
    w.vec = (double*)take(p.ws_vec);
    w.svec = (int64_t)(al256(p.ws_vec) / sizeof(double));
    w.part = (double*)take(p.ws_part);
    w.spart = (int64_t)(al256(p.ws_part) / sizeof(double));
    w.sub = (char*)take(p.ws_sub);
}

// Near-field chunk-start states of the plan: the transfer data of every
// (row, chunk) item (k_near_items without an input), then a per-row scan.
hipError_t plan_prepare(Plan& p) {
    if (p.sub) {
        hipError_t e = plan_prepare(*p.sub);
        if (e != hipSuccess) return e;
    }
    if (p.far.nterm > 0) {
        const int N = (int)p.N;
        hipError_t e = hipMalloc(&p.d_amp, (size_t)N * sizeof(cplx));
        if (e == hipSuccess) e = hipMalloc(&p.d_rowf, (size_t)N * sizeof(cplx));
        if (e != hipSuccess) return e;
        launch(k_far_tables, (N + 255) / 256, 256, 0, 0, N, p.far, p.d_amp, p.d_rowf);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
    }
    const NearParams& NP = p.near;
    if (NP.nitems <= 0) return hipSuccess;
    const int N = (int)p.N;
    // items: 8 doubles per item, later reused for the chunk-start states
    double* items = nullptr;
    hipError_t e = hipMalloc(&items, (size_t)NP.nitems * 10 * sizeof(double));
    if (e != hipSuccess) return e;
    double* st1 = items + (size_t)NP.nitems * 8;
    e = hipMalloc(&p.d_near_st, (size_t)NP.nitems * 2 * NEAR_NSUB * sizeof(double));
    if (e == hipSuccess) {
        launch(k_near_items, dim3(p.tn_wg, 1, 1), 64, 0, 0, N, NP, p.d_tn_wgseg, p.d_tn_segoff, p.d_rcp, items);
        launch(k_tnear_scan, dim3(NP.jnear, 1, 1), 64, 0, 0, NP, items, 0, st1, 0);
        launch(k_near_substates, dim3(p.tn_wg, 1, 1), 64, 0, 0, N, NP, p.d_tn_wgseg, p.d_tn_segoff, p.d_rcp, st1,
                                                           p.d_near_st);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    hipError_t e2 = hipFree(items);
    return (e != hipSuccess) ? e : e2;
}

// The batched dense block pays on the matrix cores once a tile of it is
// shared by enough instances (a block's 32 instance columns are then mostly
// live); single instances keep the one-instance kernel.
static bool dense_mm_pays(int nd, int64_t nb) { return nb >= 8 && nd >= 64; }
// Splits of the batched dense block's inner range: one (sums written
// directly) once the row and instance tiles alone give 512 blocks, else one
// per chunk of the one-instance kernels, whose partial buffer and reduction
// it then shares.
static int dense_mm_splits(int nd, int64_t nb, int nchunk) {
    const int64_t tiles = ((nb + DMM_B - 1) / DMM_B) * (((nd + 1) / 2 + DMM_I - 1) / DMM_I);
    return (tiles >= 512 || nchunk <= 1) ? 1 : nchunk;
}

// Makes `to` wait for everything enqueued on `from` so far.
static hipError_t dep(hipStream_t from, hipStream_t to, hipEvent_t e) {
    if (from == to) return hipSuccess;
    hipError_t r = hipEventRecord(e, from);
    if (r != hipSuccess) return r;
    return hipStreamWaitEvent(to, e, 0);
}

#define DLT_TRY(x)                            \
    do {                                      \
        hipError_t e_ = (x);                  \
        if (e_ != hipSuccess) return e_;      \
    } while (0)

// Boundary nodes (few, recurrence-based) and interior nodes (one thread
// each) are independent: with side streams they run side by side.
hipError_t run_nodes(const Plan& p, double* theta, double* w, double* dth, const Lanes& L) {
    trace_n = p.N;
    const NodeParams& P = p.nodes;
    const hipStream_t s = L.s, sb = L.aux(0);
    int nh = (P.N + 1) / 2;
    int ni = P.closed_b ? nh : nh - P.kb;
    if (P.kb > 0 && !P.closed_b) {
        DLT_TRY(dep(s, sb, L.ev[0]));
        int T = 64;
        while (T < 1024 && T * 256 < P.N) T *= 2;
        size_t shm = (size_t)7 * T * sizeof(double);
        traced("k_nodes_boundary", sb, [&] { launch(k_nodes_boundary, P.kb, T, shm, sb, P, p.d_guess, theta, w, dth); });
    }
    if (ni > 0)
        traced("k_nodes_interior", s, [&] { launch(k_nodes_interior, (ni + 255) / 256, 256, 0, s, P, theta, w, dth); });
    if (P.kb > 0 && !P.closed_b) DLT_TRY(dep(sb, s, L.ev[1]));
    return hipGetLastError();
}

// Scratch of a sub-plan's run: the parent's sub region.
static Work sub_work(const Plan& sub, int64_t nb, const Work& w) {
    Work sw;
    work_carve(sub, nb, (void*)w.sub, sw);
    return sw;
}

// chat = M c.  Columns n < nd: the exact conversion (dense for nd <= 8192,
// otherwise the same algorithm at size nd, recursively); columns n >= nd:
// values on the Chebyshev grid from the near and far fields, then DCT-II.
// With side streams the low block and the near field run beside the far
// field and join before the DCT-II passes that read them.
hipError_t run_leg2cheb(const Plan& p, int64_t nb, const double* c, int64_t cs, double* chat, int64_t hs, Work& w,
                        const Lanes& L) {
    trace_n = p.N;
    const int N = (int)p.N;
    const int nd = p.nd;
    const Geo& g = p.geo;
    const hipStream_t s = L.s;
    const bool last = (N <= nd);  // the dense block is the whole conversion
    const hipStream_t sl = last ? s : L.aux(1), sn = L.aux(2);
    double* dense_out = w.dense + (int64_t)p.dense_nchunk * nd;
    auto dense_block = [&](hipStream_t st, double* dst, int64_t ds) {
        if (dense_mm_pays(nd, nb)) {  // one contraction on the matrix cores
            const int zs = dense_mm_splits(nd, nb, p.dense_nchunk);
            const dim3 gm((unsigned)((nb + DMM_B - 1) / DMM_B), (unsigned)(((nd + 1) / 2 + DMM_I - 1) / DMM_I),
                          (unsigned)zs);
            if (zs == 1) {
                traced("k_dense_mm", st, [&] { launch(k_dense_mm<false>, gm, 256, 0, st, nd, p.d_lam, c, cs, (int)nb, dst, ds, 0); });
            } else {  // chunk partials, then the one-instance kernels' reduction
                traced("k_dense_mm", st, [&] {
                    launch(k_dense_mm<false>, gm, 256, 0, st, nd, p.d_lam, c, cs, (int)nb, w.dense, w.sdense, 0);
                });
                traced("k_dense_reduce", st, [&] {
                    launch(k_dense_reduce, dim3((nd + 255) / 256, 1, (unsigned)nb), 256, 0, st, nd, p.dense_nchunk,
                           p.dense_chunk, w.dense, w.sdense, dst, ds);
                });
            }
            return;
        }
        dim3 gd(2 * ((nd + 511) / 512), p.dense_nchunk, (unsigned)nb);
        traced("k_dense", st, [&] { launch(k_dense, gd, 256, 0, st, N, nd, p.dense_chunk, p.d_lam, c, cs, w.dense, w.sdense); });
        traced("k_dense_reduce", st, [&] {
            launch(k_dense_reduce, dim3((nd + 255) / 256, 1, (unsigned)nb), 256, 0, st, nd, p.dense_nchunk, p.dense_chunk,
                   w.dense, w.sdense, dst, ds);
        });
    };
    if (last) {
        dense_block(s, chat, hs);
        return hipGetLastError();
    }
    // near field (reads only c).  It is enqueued first and its end recorded
    // at once, so that a nested low-degree run can queue its own near field
    // behind it on the same stream without delaying this run's DCT.
    const NearParams& NP = p.near;
    if (!L.near_inline) DLT_TRY(dep(s, sn, L.ev[3]));
    if (NP.nitems > 0)
        traced("k_near_sums", sn, [&] {
            launch(k_near_sums, dim3(p.tn_wg, 1, (unsigned)nb), 64, 0, sn, N, NP, p.d_tn_wgseg, p.d_tn_segoff, p.d_rcp,
                                                                      p.d_near_st, c, cs, w.items, w.sitems);
        });
    if (NP.jnear > 0)
        traced("k_near_reduce", sn, [&] {
            launch(k_near_reduce, dim3(NP.jnear, 1, (unsigned)nb), 64, 0, sn, NP, w.items, w.sitems, w.near, w.snear);
        });
    if (sn != s) DLT_TRY(hipEventRecord(L.ev[4], sn));
    // low block: the dense block, or the whole method at size nd
    DLT_TRY(dep(s, sl, L.ev[2]));
    if (!p.sub) {
        dense_block(sl, dense_out, w.sdense);
    } else {
        Work sw = sub_work(*p.sub, nb, w);
        DLT_TRY(run_leg2cheb(*p.sub, nb, c, cs, dense_out, w.sdense, sw, L.nested_leg2cheb(sl)));
        trace_n = p.N;
    }
    // far field
    const FarParams& F = p.far;
    const dim3 gA(g.N1 / g.colsA, p.tgA, (unsigned)nb), gB(g.N2 / g.rowsB, p.tgB, (unsigned)nb);
    if (p.prec == PREC_FP32_BULK) {
        cplxf* X = (cplxf*)w.X;
        const int64_t sX = 2 * w.sX;
        traced("k_far_passA_f32", s, [&] {
            LEN_LAUNCH_R(g.N >= FFT_CAP, g.N2, k_far_passA, float, gA, FFT_THREADS, 0, s, g, F, p.tgA, p.d_amp, c, cs, X, sX);
        });
        traced("k_far_passB_f32", s, [&] {
            LEN_LAUNCH_R(g.N >= FFT_CAP, g.N1, k_far_passB, float, gB, FFT_THREADS, 0, s, g, F, p.tgB, p.d_rowf, X, sX, w.v, w.sv);
        });
    } else {
        traced("k_far_passA", s, [&] {
            LEN_LAUNCH_R(g.N >= FFT_CAP, g.N2, k_far_passA, double, gA, FFT_THREADS, 0, s, g, F, p.tgA, p.d_amp, c, cs, w.X, w.sX);
        });
        traced("k_far_passB", s, [&] {
            LEN_LAUNCH_R(g.N >= FFT_CAP, g.N1, k_far_passB, double, gB, FFT_THREADS, 0, s, g, F, p.tgB, p.d_rowf, w.X, w.sX, w.v, w.sv);
        });
    }
    // values on the grid -> coefficients
    if (sn != s) DLT_TRY(hipStreamWaitEvent(s, L.ev[4], 0));
    traced("k_dct2_passA", s, [&] {
        LEN_LAUNCH(g.N >= FFT_CAP, g.N2, k_dct2_passA, (dim3(g.N1 / g.colsA, 1, (unsigned)nb)), FFT_THREADS, 0, s, g, p.tgB, w.v, w.sv, w.near, w.snear,
                                                                                NP.jnear, w.X, w.sX);
    });
    DLT_TRY(dep(sl, s, L.ev[5]));
    traced("k_dct2_passB", s, [&] {
        LEN_LAUNCH(g.N >= FFT_CAP, g.N1, k_dct2_passB, (dim3(g.N2 / g.rowsB, 1, (unsigned)nb)), FFT_THREADS, 0, s, g, nd, w.X, w.sX, dense_out, w.sdense,
                                                                                chat, hs);
    });
    return hipGetLastError();
}

// out = M^T y (times n + 1/2 when `half`): rows n < nd from the exact
// conversion (dense or recursive), rows n >= nd as P^T C D_eps y on the grid.
// With side streams the low block runs beside everything else and the
// transposed near field beside the transposed far field.
hipError_t run_chebvals2cheb(const Plan& p, int64_t nb, const double* v, int64_t vs, double* chat, int64_t hs,
                             Work& w, const Lanes& L) {
    trace_n = p.N;
    const Geo& g = p.geo;
    const hipStream_t s = L.s;
    // one slab of values, no near-field rows (never read), no low block
    traced("k_dct2_passA", s, [&] {
        LEN_LAUNCH(g.N >= FFT_CAP, g.N2, k_dct2_passA, (dim3(g.N1 / g.colsA, 1, (unsigned)nb)), FFT_THREADS, 0, s, g, 1,
                   v, vs, v, vs, 0, w.X, w.sX);
    });
    traced("k_dct2_passB", s, [&] {
        LEN_LAUNCH(g.N >= FFT_CAP, g.N1, k_dct2_passB, (dim3(g.N2 / g.rowsB, 1, (unsigned)nb)), FFT_THREADS, 0, s, g, 0,
                   w.X, w.sX, v, vs, chat, hs);
    });
    return hipGetLastError();
}

hipError_t run_fill_zero(double* x, int64_t n, hipStream_t s) {
    // zero bits are 0.0: a fill kernel (no memset node in a captured graph)
    traced("k_fill_int", s, [&] { launch(k_fill_int, (unsigned)((2 * n + 255) / 256), 256, 0, s, (int*)x, 2 * n, 0); });
    return hipGetLastError();
}

hipError_t run_leg2cheb_t(const Plan& p, int64_t nb, const double* y, int64_t ys, double* out, int64_t os, int half,
                          Work& w, const Lanes& L) {
    trace_n = p.N;
    const int N = (int)p.N;
    const int nd = p.nd;
    const Geo& g = p.geo;
    const int tilesA = g.N1 / g.colsA;
    const hipStream_t s = L.s;
    const bool last = (N <= nd);
    // the transposed near field beside the transposed far field up to
    // TNEAR_SIDE_MAX_N; above it on s, before the far field (measured on one
    // box at 2^20: the far-field passes lose more to sharing the CUs with it
    // than the overlap saves, the inverse 3% faster in sequence; at 2^18 the
    // overlap is 1% faster)
    const hipStream_t sl = last ? s : L.aux(1), sn = (p.N <= TNEAR_SIDE_MAX_N) ? L.aux(2) : s;
    double* dense_out = w.dense + (int64_t)p.dense_nchunk * nd;
    if (!L.low_inline) DLT_TRY(dep(s, sl, L.ev[6]));
    if (!p.sub && dense_mm_pays(nd, nb)) {  // one contraction on the matrix cores
        double* dst = last ? out : dense_out;
        const int64_t ds = last ? os : w.sdense;
        const int zs = dense_mm_splits(nd, nb, p.dense_nchunk);
        const dim3 gm((unsigned)((nb + DMM_B - 1) / DMM_B), (unsigned)(((nd + 1) / 2 + DMM_I - 1) / DMM_I), (unsigned)zs);
        if (zs == 1) {
            traced("k_dense_mm_t", sl, [&] {
                launch(k_dense_mm<true>, gm, 256, 0, sl, nd, p.d_lam, y, ys, (int)nb, dst, ds, last ? half : 0);
            });
        } else {  // chunk partials, then the one-instance kernels' reduction
            traced("k_dense_mm_t", sl, [&] {
                launch(k_dense_mm<true>, gm, 256, 0, sl, nd, p.d_lam, y, ys, (int)nb, w.dense, w.sdense, 0);
            });
            traced("k_dense_t_reduce", sl, [&] {
                launch(k_dense_t_reduce, dim3((nd + 255) / 256, 1, (unsigned)nb), 256, 0, sl, nd, p.dense_nchunk,
                       p.dense_chunk, w.dense, w.sdense, dst, ds, last ? half : 0);
            });
        }
        if (last) return hipGetLastError();
    } else if (!p.sub) {
        traced("k_dense_t", sl, [&] {
            launch(k_dense_t, dim3(2 * ((nd + 511) / 512), p.dense_nchunk, (unsigned)nb), 256, 0, sl, nd, p.dense_chunk, p.d_lam,
                                                                                          y, ys, w.dense, w.sdense);
        });
        double* dst = last ? out : dense_out;
        int64_t ds = last ? os : w.sdense;
        int hf = last ? half : 0;
        traced("k_dense_t_reduce", sl, [&] {
            launch(k_dense_t_reduce, dim3((nd + 255) / 256, 1, (unsigned)nb), 256, 0, sl, nd, p.dense_nchunk, p.dense_chunk,
                                                                                  w.dense, w.sdense, dst, ds, hf);
        });
        if (last) return hipGetLastError();
    } else {
        Work sw = sub_work(*p.sub, nb, w);
        // the nested run's low block beside its other passes, from N = 2^18
        // down (measured on one box: the 2^18 inverse 3.5% faster; at 2^20
        // the extra concurrency slows the transposed far field and the
        // inverse by 4%, so there the nested run stays on one stream)
        const Lanes NL = (p.N <= NESTED_LOW_MAX_N) ? L.nested_leg2cheb_t(sl) : L.on(sl);
        if (NL.low_inline) DLT_TRY(dep(s, NL.side[1], L.ev[16]));  // the nested run's low-block stream
        DLT_TRY(run_leg2cheb_t(*p.sub, nb, y, ys, dense_out, w.sdense, 0, sw, NL));
        trace_n = p.N;
    }
    const NearParams& NP = p.near;
    // u = C D_eps y on the grid
    double* u = w.vec;
    traced("k_dct3_passA", s, [&] {
        LEN_LAUNCH(g.N >= FFT_CAP, g.N2, k_dct3_passA, (dim3(tilesA, 1, (unsigned)nb)), FFT_THREADS, 0, s, g, y, ys, w.X, w.sX);
    });
    traced("k_dct3_passB", s, [&] {
        LEN_LAUNCH(g.N >= FFT_CAP, g.N1, k_dct3_passB, (dim3(g.N2 / g.rowsB, 1, (unsigned)nb)), FFT_THREADS, 0, s, g, w.X, w.sX, u, w.svec);
    });
    // transposed near field
    DLT_TRY(dep(s, sn, L.ev[7]));
    if (NP.nitems > 0) {
        traced("k_tnear_accum", sn, [&] {
            launch(k_tnear_accum, dim3(p.tn_wg, 1, (unsigned)nb), 64, 0, sn, N, NP, p.d_tn_wgseg, p.d_tn_segoff, p.d_rcp, u,
                                                                        w.svec, p.d_near_st, w.part, w.spart);
        });
    }
    // transposed far field
    const dim3 gA(tilesA, p.tgA, (unsigned)nb), gB(g.N2 / g.rowsB, p.tgB, (unsigned)nb);
    if (p.prec == PREC_FP32_BULK) {
        cplxf* X = (cplxf*)w.X;
        const int64_t sX = 2 * w.sX;
        traced("k_tfar_passA_f32", s, [&] {
            LEN_LAUNCH_R(g.N >= FFT_CAP, g.N2, k_tfar_passA, float, gA, FFT_THREADS, 0, s, g, p.far, p.tgA, p.d_rowf, u, w.svec, X, sX);
        });
        traced("k_tfar_passB_f32", s, [&] {
            LEN_LAUNCH_R(g.N >= FFT_CAP, g.N1, k_tfar_passB, float, gB, FFT_THREADS, 0, s, g, p.far, p.tgB, p.d_amp, X, sX, w.v, w.sv);
        });
    } else {
        traced("k_tfar_passA", s, [&] {
            LEN_LAUNCH_R(g.N >= FFT_CAP, g.N2, k_tfar_passA, double, gA, FFT_THREADS, 0, s, g, p.far, p.tgA, p.d_rowf, u, w.svec, w.X, w.sX);
        });
        traced("k_tfar_passB", s, [&] {
            LEN_LAUNCH_R(g.N >= FFT_CAP, g.N1, k_tfar_passB, double, gB, FFT_THREADS, 0, s, g, p.far, p.tgB, p.d_amp, w.X, w.sX, w.v, w.sv);
        });
    }
    DLT_TRY(dep(sn, s, L.ev[8]));
    DLT_TRY(dep(sl, s, L.ev[9]));
    traced("k_idlt_final", s, [&] {
        launch(k_idlt_final, dim3((N + 255) / 256, 1, (unsigned)nb), 256, 0, s, N, nd, (NP.nitems > 0) ? p.tn_nrg : 0,
                                                                          p.d_tn_rgnend, dense_out, w.sdense, p.tgB, w.v,
                                                                          w.sv, w.part, w.spart, out, os, half);
    });
    return hipGetLastError();
}

// Pair groups of an FP64 Taylor pass A (grid rows, each taking an equal
// share of the pairs) over `tiles` tile blocks: the fewest that give the
// launch 256 blocks.  Measured on one box, pass A and its transpose at
// N = 2^20 (512 tiles) are fastest with one group (two and four groups:
// 20% and 60% slower), at 2^18 (128 tiles) with two (eight: 23% slower),
// at 2^16 and below with one pair per group.
static int pass_a_groups(int64_t tiles, int npairs) {
    int qg = 1;
    while (qg < npairs && tiles * qg < 256) ++qg;
    return qg;
}

hipError_t run_ndct(const Plan& p, int64_t nb, const double* chat, int64_t hs, const double* dth, double* f,
                    Work& w, const Lanes& L, const RaggedRows* rr, int Qo) {
    trace_n = p.N;
    const Geo& g = p.geo;
    const hipStream_t s = L.s;
    const int Q = Qo > 0 ? Qo : p.L / 2;
    const RaggedRows RR = rr ? *rr : RaggedRows{nullptr, nullptr, nullptr, nullptr};
    const int tilesA = g.N1 / g.colsA;
    const int N = (int)p.N;
    const dim3 gB(g.N2 / g.rowsB, 1, (unsigned)nb);
    if (p.prec == PREC_FP32_BULK) {
        // pair 0 in FP64 (slab 0 of X), pairs 1..Q-1 in FP32 behind it
        cplxf* X1 = (cplxf*)(w.X + N);
        const int64_t s1 = 2 * w.sX;
        const int QG = (tilesA * nb >= 256) ? 1 : std::max(Q - 1, 1);
        // pair 0 (FP64) on the first side stream beside pairs 1..Q-1 (FP32):
        // both read chat and write separate slabs (measured on one box: the
        // FP32-bulk forward at 2^20, batch 64, 3% faster; the same in the
        // inverse's transposed pass A gained nothing and is not used)
        const hipStream_t s0 = L.aux(0);
        DLT_TRY(dep(s, s0, L.ev[10]));
        traced("k_ndct_passA", s0, [&] {
            LEN_LAUNCH(g.N >= FFT_CAP, g.N2, k_ndct_pair, (dim3(tilesA, 1, (unsigned)nb)), FFT_THREADS, 0, s0, g, 0, chat, hs, w.X, w.sX);
        });
        if (Q > 1)
            traced("k_ndct_passA_f32", s, [&] {
                LEN_LAUNCH_R(g.N >= FFT_CAP, g.N2, k_ndct_passA, float, (dim3(tilesA, QG, (unsigned)nb)), FFT_THREADS, 0, s, g, 1, Q, QG, chat, hs, X1, s1);
            });
        DLT_TRY(dep(s0, s, L.ev[11]));
        traced("k_ndct_passB_f32", s, [&] {
            LEN_LAUNCH_R(g.N >= FFT_CAP, g.N1, k_ndct_passB, float, gB, FFT_THREADS, 0, s, g, Q, w.X, w.sX, X1, s1, dth, f, p.N, RR);
        });
    } else {
        const int QG = pass_a_groups(tilesA * nb, Q);
        traced("k_ndct_passA", s, [&] {
            if (QG == Q)  // one pair per group
                LEN_LAUNCH(g.N >= FFT_CAP, g.N2, k_ndct_pair, (dim3(tilesA, QG, (unsigned)nb)), FFT_THREADS, 0, s, g, 0, chat, hs, w.X, w.sX);
            else
                LEN_LAUNCH_R(g.N >= FFT_CAP, g.N2, k_ndct_passA, double, (dim3(tilesA, QG, (unsigned)nb)), FFT_THREADS, 0, s, g, 0, Q, QG, chat, hs, w.X, w.sX);
        });
        traced("k_ndct_passB", s, [&] {
            LEN_LAUNCH_R(g.N >= FFT_CAP, g.N1, k_ndct_passB, double, gB, FFT_THREADS, 0, s, g, Q, w.X, w.sX, w.X + N, w.sX, dth, f, p.N, RR);
        });
    }
    return hipGetLastError();
}

// H = F^+(cyclic chirp)/M of the theta^cheb* plan, formed once on the device
hipError_t star_prepare(StarPlan& sp) {
    const Geo& g = sp.geo;
    const int M = g.N;
    hipError_t e = hipMalloc(&sp.d_H, (size_t)M * sizeof(cplx));
    if (e != hipSuccess) return e;
    const int tilesA = g.N1 / g.colsA, tilesB = g.N2 / g.rowsB;
    LEN_LAUNCH(M >= FFT_CAP, g.N2, k_star_passA, dim3(tilesA, 1, 1), FFT_THREADS, 0, 0, g, (int)sp.N, 0, 1, 1, 1,
               (const double*)nullptr, (int64_t)0, (const double*)nullptr, (const double*)nullptr, sp.d_H, (int64_t)0);
    LEN_LAUNCH(M >= FFT_CAP, g.N1, k_star_passB, dim3(tilesB, 1, 1), FFT_THREADS, 0, 0, g, 1, 1, (const cplx*)nullptr,
               sp.d_H, (int64_t)0);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e;
}

// f = the expansions chat (nb instances, stride hs) at the Legendre nodes by
// the Taylor series about theta^cheb*, or with wts (the transposed
// evaluation) y = T^T (wts * in) into f; X: nb x L slabs of M values
hipError_t run_star(const StarPlan& sp, int64_t nb, const double* chat, int64_t hs, const double* wts,
                    const double* dth, double* f, int64_t fs, cplx* X, hipStream_t s) {
    trace_n = sp.N;
    const Geo& g = sp.geo;
    const int M = g.N;
    const int L = sp.L;
    const int tilesA = g.N1 / g.colsA, tilesB = g.N2 / g.rowsB;
    // small transforms: split the terms over blocks for parallelism
    const int QG = (tilesA * nb >= 256) ? 1 : L;
    const int64_t xs = (int64_t)L * M;
    traced("k_star_passA", s, [&] {
        LEN_LAUNCH(M >= FFT_CAP, g.N2, k_star_passA, dim3(tilesA, QG, (unsigned)nb), FFT_THREADS, 0, s, g, (int)sp.N, 0,
                   L, QG, wts ? 2 : 0, chat, hs, wts, dth, X, xs);
    });
    traced("k_star_passB", s, [&] {
        LEN_LAUNCH(M >= FFT_CAP, g.N1, k_star_passB, dim3(tilesB, 1, (unsigned)nb), FFT_THREADS, 0, s, g, L, 0,
                   (const cplx*)sp.d_H, X, xs);
    });
    traced("k_star_passC", s, [&] {
        LEN_LAUNCH(M >= FFT_CAP, g.N2, k_star_passC, dim3(tilesA, 1, (unsigned)nb), FFT_THREADS, 0, s, g, (int)sp.N, L,
                   wts ? 1 : 0, (const cplx*)X, xs, dth, f, fs);
    });
    return hipGetLastError();
}

hipError_t run_inverse(const Plan& p, int64_t nb, const double* f, const double* wts, const double* dth,
                       double* c, Work& w, const Lanes& L, const RaggedRows* rr, int Qo) {
    trace_n = p.N;
    const int N = (int)p.N;
    const Geo& g = p.geo;
    const hipStream_t s = L.s;
    const int Q = Qo > 0 ? Qo : p.L / 2;
    const RaggedRows RR = rr ? *rr : RaggedRows{nullptr, nullptr, nullptr, nullptr};
    const int tilesA = g.N1 / g.colsA;
    double* y = w.chat;  // T^T D_w f, stride w.schat
    const int tilesB = (g.N2 == 1) ? 1 : g.N2 / g.rowsB;
    const dim3 gB(tilesB, 1, (unsigned)nb);
    if (p.prec == PREC_FP32_BULK) {
        cplxf* X1 = (cplxf*)(w.X + N);
        const int64_t s1 = 2 * w.sX;
        const int QG = (tilesA * nb >= 256) ? 1 : std::max(Q - 1, 1);
        traced("k_tndct_passA", s, [&] {
            LEN_LAUNCH(g.N >= FFT_CAP, g.N2, k_tndct_pair, (dim3(tilesA, 1, (unsigned)nb)), FFT_THREADS, 0, s, g, 0, f, N, wts, dth, w.X, w.sX, RR);
        });
        if (Q > 1)
            traced("k_tndct_passA_f32", s, [&] {
                LEN_LAUNCH_R(g.N >= FFT_CAP, g.N2, k_tndct_passA, float, (dim3(tilesA, QG, (unsigned)nb)), FFT_THREADS, 0, s, g, 1, Q, QG, f, N, wts, dth, X1, s1, RR);
            });
        traced("k_tndct_passB_f32", s, [&] {
            LEN_LAUNCH_R(g.N >= FFT_CAP, g.N1, k_tndct_passB, float, gB, FFT_THREADS, 0, s, g, Q, w.X, w.sX, X1, s1, y, w.schat);
        });
    } else {
        const int QG = pass_a_groups(tilesA * nb, Q);
        traced("k_tndct_passA", s, [&] {
            if (QG == Q)  // one pair per group
                LEN_LAUNCH(g.N >= FFT_CAP, g.N2, k_tndct_pair, (dim3(tilesA, QG, (unsigned)nb)), FFT_THREADS, 0, s, g, 0, f, N, wts, dth, w.X, w.sX, RR);
            else
                LEN_LAUNCH_R(g.N >= FFT_CAP, g.N2, k_tndct_passA, double, (dim3(tilesA, QG, (unsigned)nb)), FFT_THREADS, 0, s, g, 0, Q, QG, f, N, wts, dth, w.X, w.sX, RR);
        });
        traced("k_tndct_passB", s, [&] {
            LEN_LAUNCH_R(g.N >= FFT_CAP, g.N1, k_tndct_passB, double, gB, FFT_THREADS, 0, s, g, Q, w.X, w.sX, w.X + N, w.sX, y, w.schat);
        });
    }
    return run_leg2cheb_t(p, nb, y, w.schat, c, N, 1, w, L);
}

hipError_t run_rnodes(const RaggedNodes& rn, int Ng, int* gk, double* dg, double* wg, double* theta, double* w,
                      double* dth, hipStream_t s) {
    trace_n = Ng;
    if (gk) {
        const int64_t n = (int64_t)rn.nb * Ng;
        traced("k_fill_int", s, [&] { launch(k_fill_int, (unsigned)((n + 255) / 256), 256, 0, s, gk, n, -1); });
    }
    if (rn.nbnd_total > 0) {
        if (Ng <= RNODE_THREAD_MAX_NG) {  // short recurrences: one thread per node
            traced("k_rnodes_bthread", s, [&] {
                launch(k_rnodes_bthread, (rn.nbnd_total + 255) / 256, 256, 0, s, rn.R, rn.boff, rn.nb, Ng, gk, dg, wg,
                       theta, w, dth);
            });
        } else {
            traced("k_rnodes_boundary", s, [&] {
                launch(k_rnodes_boundary, rn.nbnd_total, 256, 0, s, rn.R, rn.boff, rn.nb, Ng, gk, dg, wg, theta, w, dth);
            });
        }
    }
    if (rn.ni_total > 0)
        traced("k_rnodes_interior", s, [&] {
            launch(k_rnodes_interior, (rn.ni_total + 255) / 256, 256, 0, s, rn.R, rn.ioff, rn.nb, Ng, gk, dg, wg, theta, w,
                                                                       dth);
        });
    return hipGetLastError();
}

hipError_t run_rgather(const double* in, const RNode* R, const int64_t* offs, int nb, int Ng, int64_t stride,
                       double* out, hipStream_t s) {
    trace_n = Ng;
    traced("k_rgather", s, [&] { launch(k_rgather, dim3((Ng + 255) / 256, nb), 256, 0, s, in, R, offs, Ng, stride, out); });
    return hipGetLastError();
}

hipError_t run_rscatter(const double* in, int64_t stride, const RNode* R, const int64_t* offs, int nb, int Ng,
                        double* out, hipStream_t s) {
    trace_n = Ng;
    traced("k_rscatter", s, [&] { launch(k_rscatter, dim3((Ng + 255) / 256, nb), 256, 0, s, in, stride, R, offs, out); });
    return hipGetLastError();
}

}  // namespace dlt
