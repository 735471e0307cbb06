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

// ------------------------------------------------------------------ nodes --
// Interior nodes k in [kb, ceil(N/2)): Newton in delta = theta - theta*_k
// (theta*_k = (k+1/2)pi/N) on the M-term Stieltjes expansion of P_N(cos theta)
// with the large phase (N+m+1/2) theta reduced exactly:
//   (N+m+1/2) theta*_k - (m+1/2) pi/2 = (k+1/2) pi + (m+1/2)(theta*_k - pi/2),
// so cos(phase) = -(-1)^k sin psi_m, sin(phase) = (-1)^k cos psi_m with
// psi_m = (m+1/2)(theta - pi/2) + N delta.
__global__ void k_nodes_interior(NodeParams P, double* __restrict__ theta, double* __restrict__ w,
                                 double* __restrict__ dth) {
    const int N = P.N;
    const int nh = (N + 1) / 2;
    int k = P.kb + blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nh) return;
    const double pi = 3.141592653589793;
    // theta^cheb* - theta^cheb1 = pi (N - 2k - 1) / (4 N (N + 1/2))
    double delta = pi * (double)(N - 2 * k - 1) / (4.0 * N * (N + 0.5));
    // theta*_k - pi/2 = pi (2k + 1 - N) / (2N)
    const double a0 = pi * (double)(2 * k + 1 - N) / (2.0 * N);
    const double ts = (k + 0.5) * pi / N;
    double Pv = 0, Dv = 0, s2 = 1;
    for (int it = 0; it <= 5; ++it) {
        double th = ts + delta;
        double sn, cs;
        sincos(th, &sn, &cs);
        s2 = 2.0 * sn;
        double cot = cs / sn;
        double q = 1.0 / s2;
        // psi_0 and the per-term increment theta - pi/2
        double dlt = a0 + delta;  // theta - pi/2
        double ps, pc, rs, rc;
        sincos(0.5 * dlt + N * delta, &ps, &pc);
        sincos(dlt, &rs, &rc);
        double r = sqrt(q);
        Pv = 0;
        Dv = 0;
#pragma unroll 4
        for (int m = 0; m < P.Ms; ++m) {
            double hm = P.h[m] * r;
            Pv = fma(hm, ps, Pv);
            Dv = fma(hm, (N + m + 0.5) * pc - (m + 0.5) * ps * cot, Dv);
            // psi_{m+1} = psi_m + (theta - pi/2)
            double nps = ps * rc + pc * rs;
            double npc = pc * rc - ps * rs;
            ps = nps;
            pc = npc;
            r *= q;
        }
        if (it < 5) delta -= Pv / Dv;
    }
    // dP/dtheta = -(-1)^k C D;  w = 2 / (dP/dtheta)^2
    double dP = P.C * Dv;
    double wk = 2.0 / (dP * dP);
    double th = ts + delta;
    int k2 = N - 1 - k;
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

// P_N(cos t), P_{N-1}(cos t) and the Christoffel sum K = sum_{n<N} (2n+1) P_n^2
// for 0 < t <= pi/2, by the recurrence in u = 2 sin^2(t/2),
//   D_{n+1} = (n D_n - (2n+1) u P_n)/(n+1),  P_{n+1} = P_n + D_{n+1},
// split over the block: each thread runs its chunk of degrees for the two
// basis states (P, D) = (1, 0) and (0, 1) (the first chunk from the true
// start), keeping the chunk's transfer matrix and the quadratic sums
// sum (2n+1) Pa^2, sum (2n+1) Pa Pb, sum (2n+1) Pb^2; the chunks are then
// chained in order.  `sh` holds 7*blockDim.x + 3 doubles.
__device__ void block_legendre_pair(int N, double t, const double* __restrict__ A,
                                    const double* __restrict__ B, double* sh, double* pN, double* pN1,
                                    double* kc) {
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
        double bu = B[n] * u;
        double dna = fma(A[n], da, -bu * pa);
        double dnb = fma(A[n], db, -bu * pb);
        pa += dna;
        da = dna;
        pb += dnb;
        db = dnb;
    }
    double* q = sh + 7 * tid;
    q[0] = pa;
    q[1] = da;
    q[2] = pb;
    q[3] = db;
    q[4] = saa;
    q[5] = sab;
    q[6] = sbb;
    __syncthreads();
    if (tid == 0) {
        double P = 1, D = 0, K = 0;  // state at n = 0 (D_0 does not enter)
        int nthr = min(T, (N + C - 1) / C);
        for (int i = 0; i < nthr; ++i) {
            const double* r = sh + 7 * i;
            K += P * P * r[4] + 2.0 * P * D * r[5] + D * D * r[6];
            double Pn = r[0] * P + r[2] * D;
            double Dn = r[1] * P + r[3] * D;
            P = Pn;
            D = Dn;
        }
        sh[7 * T] = P;
        sh[7 * T + 1] = P - D;
        sh[7 * T + 2] = K;
    }
    __syncthreads();
    *pN = sh[7 * T];
    *pN1 = sh[7 * T + 1];
    *kc = sh[7 * T + 2];
    __syncthreads();
}

// Boundary nodes k < kb.  The start `guess` (offset from theta*_k) is the
// Bessel-zero form theta ~ psi + (psi cot psi - 1)/(8 psi nu^2), psi =
// j_{0,k+1}/nu, nu = N + 1/2, whose error is O(nu^-4) (one ulp from
// N = 4096 on), or theta^cheb* for small N; `newton_b` Newton steps with the
// exact recurrence follow (none for large N, where the FP64 recurrence is
// less accurate than the start).  The weight is the Christoffel number
// w_k = 2 / sum_{n<N} (2n+1) P_n(x_k)^2, which is well conditioned in x_k.
__global__ void k_nodes_boundary(NodeParams P, const double* __restrict__ guess, const double* __restrict__ A,
                                 const double* __restrict__ B, double* __restrict__ theta,
                                 double* __restrict__ w, double* __restrict__ dth) {
    extern __shared__ double sh[];
    const int N = P.N;
    const int k = blockIdx.x;
    const double pi = 3.141592653589793;
    const double ts = (k + 0.5) * pi / N;
    double delta = guess[k];
    double pN, pN1, kc;
    const bool middle = (N & 1) && (k == (N - 1) / 2);
    if (middle) {
        delta = 0;  // x = 0 is a root of odd-degree P_N and theta*_k = pi/2 there
    } else {
        for (int it = 0; it < P.newton_b; ++it) {
            double th = ts + delta;
            block_legendre_pair(N, th, A, B, sh, &pN, &pN1, &kc);
            double sn, cs;
            sincos(th, &sn, &cs);
            double dP = N * (cs * pN - pN1) / sn;
            double step = pN / dP;
            delta -= step;
            if (fabs(step) <= 2.2e-16 * th) break;  // uniform across the block
        }
    }
    double th = ts + delta;
    block_legendre_pair(N, th, A, B, sh, &pN, &pN1, &kc);
    if (threadIdx.x == 0) {
        double wk = 2.0 / kc;
        int k2 = N - 1 - k;
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
}

// ------------------------------------------------------------------ dense --
// chat_k (k < nd) partial sums over column chunk blockIdx.y:
//   sum_{n in chunk, n >= k, n+k even} (eps_k/pi) Lam((n-k)/2) Lam((n+k)/2) c_n
__global__ void k_dense(int N, int nd, int chunk, const double* __restrict__ lam, const double* __restrict__ c,
                        int64_t c_stride, double* __restrict__ part, int64_t part_stride) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    int ch = blockIdx.y;
    int b = blockIdx.z;
    const double* cb = c + b * c_stride;
    double* pb = part + b * part_stride;
    if (k >= nd) return;
    int n0 = ch * chunk, n1 = min(nd, n0 + chunk);
    double acc = 0;
    int n = max(n0, k);
    if ((n - k) & 1) ++n;
    for (; n < n1; n += 2) acc = fma(lam[(n - k) >> 1] * lam[(n + k) >> 1], cb[n], acc);
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

// ------------------------------------------------------ FFT pass helpers --
// Pass A: the block owns columns n_a in [na0, na0+colsA); element e of the
// tile is (col = e % colsA, n_b = e / colsA), n = na0 + col + N1 n_b.
// After the in-LDS length-N2 DFTs the tile holds buf[col*N2 + j_b]; it is
// multiplied by e^{2 pi i n_a j_b / N} and written to X[n_a*N2 + j_b].
__device__ __forceinline__ void passA_store(const Geo& g, const cplx* buf, int na0, cplx* __restrict__ X) {
    const int tot = g.colsA * g.N2;
    for (int e = threadIdx.x; e < tot; e += FFT_THREADS) {
        int col = e / g.N2, jb = e - col * g.N2;
        int na = na0 + col;
        cplx v = buf[e];
        if (na && jb) v = cmul(v, tw2(g.twHi, g.twLo, (int64_t)na * jb, g.sh));
        X[(int64_t)na * g.N2 + jb] = v;
    }
}

// Pass B: the block owns rows j_b in [jb0, jb0+rowsB); LDS holds
// buf[r*N1 + n_a]; after the length-N1 DFTs, buf[r*N1 + j_a] is output
// m = jb0 + r + N2 j_a.
__device__ __forceinline__ void passB_load(const Geo& g, cplx* buf, int jb0, const cplx* __restrict__ X) {
    const int tot = g.rowsB * g.N1;
    for (int e = threadIdx.x; e < tot; e += FFT_THREADS) {
        int r = e % g.rowsB, na = e / g.rowsB;
        buf[r * g.N1 + na] = X[(int64_t)na * g.N2 + jb0 + r];
    }
}

// ---------------------------------------------------------- far field A --
// For every term t = (block b, m), in descending m so that
// h_{m-1,n} = h_{m,n} m (n+m+1/2)/(m-1/2)^2 needs no division, the DFT input
//   b_n = C_n h_{m,n} c_n e^{i pi n/(2N)} [n >= nlo_b]
// goes through pass A of the length-N DFT.
__global__ __launch_bounds__(FFT_THREADS) void k_far_passA(Geo g, FarParams F, const double* __restrict__ c,
                                                          int64_t c_stride, cplx* __restrict__ X,
                                                          int64_t x_stride) {
    __shared__ cplx buf[FFT_CAP];
    const int N = g.N;
    const int na0 = blockIdx.x * g.colsA;
    const int b = blockIdx.z;
    const double* cb = c + b * c_stride;
    cplx* Xb = X + b * x_stride;
    const int tot = g.colsA * g.N2;
    cplx base[FFT_VPT];
    double h[FFT_VPT];
    int nn[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        int e = threadIdx.x + s * FFT_THREADS;
        base[s] = {0, 0};
        h[s] = 0;
        nn[s] = -1;
        if (e < tot) {
            int col = e % g.colsA, nb = e / g.colsA;
            int n = na0 + col + g.N1 * nb;
            nn[s] = n;
            if (n >= F.nd) {
                double amp = stieltjes_C((double)n) * cb[n];
                base[s] = cscale(half_shift(n, N), amp);
                // h_{Mmax-1,n} = prod_{j<Mmax} (j-1/2)^2/(j (n+j+1/2))
                double hv = 1;
                for (int j = 1; j < F.Mmax; ++j) hv *= (j - 0.5) * (j - 0.5) / (j * (n + j + 0.5));
                h[s] = hv;
            }
        }
    }
    for (int m = F.Mmax - 1; m >= 0; --m) {
        for (int t = 0; t < F.nterm; ++t) {
            if (F.term_m[t] != m) continue;
            const int nlo = F.blk[F.term_blk[t]].nlo;
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) {
                int e = threadIdx.x + s * FFT_THREADS;
                if (e < tot) {
                    int col = e % g.colsA, nb = e / g.colsA;
                    double f = (nn[s] >= nlo) ? h[s] : 0.0;
                    buf[col * g.N2 + nb] = cscale(base[s], f);
                }
            }
            __syncthreads();
            lds_fft(buf, g.N2, g.colsA, g.twN2);
            passA_store(g, buf, na0, Xb + (int64_t)t * N);
            __syncthreads();
        }
        if (m > 0) {
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s)
                if (nn[s] >= 0) h[s] *= m * (nn[s] + m + 0.5) / ((m - 0.5) * (m - 0.5));
        }
    }
}

// ---------------------------------------------------------- far field B --
// For every term the z-values z_j = sum_n b_n e^{i n theta_j} (z = V_m or
// conj(V_m) at row j(m)) are combined into
//   v_j += Re(e^{i (m+1/2)(theta_j - pi/2)} z_j) / (2 sin theta_j)^{m+1/2}
// on the rows of the term's block.  Term group blockIdx.y handles terms
// t = y, y + G, ...; partial values go to v[y].
__device__ __forceinline__ int row_block(const FarParams& F, int j, int N) {
    int jj = min(j, N - 1 - j);
    for (int b = 0; b < F.nblk; ++b)
        if (jj >= F.blk[b].jlo && jj < F.blk[b].jhi) return b;
    return -1;
}

__global__ __launch_bounds__(FFT_THREADS) void k_far_passB(Geo g, FarParams F, int G, const cplx* __restrict__ X,
                                                          int64_t x_stride, double* __restrict__ v,
                                                          int64_t v_stride) {
    __shared__ cplx buf[FFT_CAP];
    const int N = g.N;
    const int jb0 = blockIdx.x * g.rowsB;
    const int grp = blockIdx.y;
    const int b = blockIdx.z;
    const cplx* Xb = X + b * x_stride;
    const int tot = g.rowsB * g.N1;
    const double pi = 3.141592653589793;
    cplx gm[FFT_VPT], rq[FFT_VPT];
    double acc[FFT_VPT];
    int blk[FFT_VPT];
    bool cj[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        int e = threadIdx.x + s * FFT_THREADS;
        acc[s] = 0;
        blk[s] = -1;
        cj[s] = false;
        gm[s] = {0, 0};
        rq[s] = {0, 0};
        if (e < tot) {
            int r = e / g.N1, ja = e - r * g.N1;
            int m = jb0 + r + g.N2 * ja;
            int j = row_of(m, N);
            cj[s] = (2 * m >= N);
            blk[s] = row_block(F, j, N);
            double d = pi * (double)(2 * j + 1 - N) / (2.0 * N);  // theta_j - pi/2
            int jj = min(j, N - 1 - j);
            double sn = sin((jj + 0.5) * pi / N);                 // sin theta_j, full relative accuracy
            double q = 1.0 / (2.0 * sn);
            double ps, pc, rs, rc;
            sincos(0.5 * d, &ps, &pc);
            sincos(d, &rs, &rc);
            double r0 = sqrt(q);
            gm[s] = {pc * r0, ps * r0};
            rq[s] = {rc * q, rs * q};
        }
    }
    for (int m = 0; m < F.Mmax; ++m) {
        for (int t = 0; t < F.nterm; ++t) {
            if (F.term_m[t] != m || (t % G) != grp) continue;
            const int tb = F.term_blk[t];
            passB_load(g, buf, jb0, Xb + (int64_t)t * N);
            __syncthreads();
            lds_fft(buf, g.N1, g.rowsB, g.twN1);
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) {
                int e = threadIdx.x + s * FFT_THREADS;
                if (e < tot && blk[s] == tb) {
                    cplx z = buf[e];
                    if (cj[s]) z.im = -z.im;
                    acc[s] = fma(gm[s].re, z.re, fma(-gm[s].im, z.im, acc[s]));
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) gm[s] = cmul(gm[s], rq[s]);
    }
    double* vb = v + b * v_stride + (int64_t)grp * N;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        int e = threadIdx.x + s * FFT_THREADS;
        if (e < tot) {
            int r = e / g.N1, ja = e - r * g.N1;
            int m = jb0 + r + g.N2 * ja;
            vb[row_of(m, N)] = acc[s];
        }
    }
}

// ------------------------------------------------------------ near field --
// Item = (row j, degree chunk): the recurrence over the chunk from two basis
// states (chunk > 0) or the true start (chunk 0), accumulating
//   S+ = sum c_n P_n(cos theta_j), S- = sum (-1)^n c_n P_n(cos theta_j)
// over n >= nd; the mirror row N-1-j takes S- since P_n(-x) = (-1)^n P_n(x).
__global__ void k_near_items(int N, NearParams NP, const double* __restrict__ A, const double* __restrict__ B,
                             const double* __restrict__ c, int64_t c_stride, double* __restrict__ items,
                             int64_t it_stride) {
    int id = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.z;
    if (id >= NP.nitems) return;
    int sgi = 0;
    while (sgi + 1 < NP.nseg && id >= NP.seg[sgi + 1].item_off) ++sgi;
    const Seg S = NP.seg[sgi];
    int loc = id - S.item_off;
    int nrows = S.jhi - S.jlo;
    int ch = loc / nrows;
    int j = S.jlo + (loc - ch * nrows);
    const double* cb = c ? c + b * c_stride : nullptr;
    double* out = items + b * it_stride + (int64_t)id * 8;
    const double pi = 3.141592653589793;
    double sn = sin(0.5 * (j + 0.5) * pi / N);
    double u = 2.0 * sn * sn;
    int n0 = ch * NEAR_CHUNK, n1 = min(S.nend, n0 + NEAR_CHUNK);
    if (ch == 0) {
        double p = 1, d = 0, sp = 0, sm = 0;
        for (int n = n0; n < n1; ++n) {
            if (cb && n >= NP.nd) {
                double cn = cb[n];
                sp = fma(cn, p, sp);
                sm = fma((n & 1) ? -cn : cn, p, sm);
            }
            double dn = fma(A[n], d, -B[n] * u * p);
            p += dn;
            d = dn;
        }
        out[0] = p;
        out[1] = d;
        out[2] = sp;
        out[3] = sm;
    } else {
        double pa = 1, da = 0, pb = 0, db = 1;
        double spa = 0, spb = 0, sma = 0, smb = 0;
        for (int n = n0; n < n1; ++n) {
            if (cb && n >= NP.nd) {
                double cn = cb[n];
                double cm = (n & 1) ? -cn : cn;
                spa = fma(cn, pa, spa);
                spb = fma(cn, pb, spb);
                sma = fma(cm, pa, sma);
                smb = fma(cm, pb, smb);
            }
            double bu = B[n] * u;
            double dna = fma(A[n], da, -bu * pa);
            double dnb = fma(A[n], db, -bu * pb);
            pa += dna;
            da = dna;
            pb += dnb;
            db = dnb;
        }
        out[0] = pa;
        out[1] = da;
        out[2] = pb;
        out[3] = db;
        out[4] = spa;
        out[5] = spb;
        out[6] = sma;
        out[7] = smb;
    }
}

// near[j] = S+ for row j < jnear, near[jnear + j] = S- (row N-1-j)
__global__ void k_near_combine(NearParams NP, const double* __restrict__ items, int64_t it_stride,
                               double* __restrict__ near, int64_t near_stride) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.z;
    if (j >= NP.jnear) return;
    const double* it = items + b * it_stride;
    double* nb = near + b * near_stride;
    int sgi = -1;
    for (int s = 0; s < NP.nseg; ++s)
        if (j >= NP.seg[s].jlo && j < NP.seg[s].jhi) sgi = s;
    double sp = 0, sm = 0;
    if (sgi >= 0) {
        const Seg S = NP.seg[sgi];
        int nrows = S.jhi - S.jlo;
        const double* o = it + (int64_t)(S.item_off + (j - S.jlo)) * 8;
        double P = o[0], D = o[1];
        sp = o[2];
        sm = o[3];
        for (int ch = 1; ch < S.nchunk; ++ch) {
            const double* q = it + (int64_t)(S.item_off + ch * nrows + (j - S.jlo)) * 8;
            sp += P * q[4] + D * q[5];
            sm += P * q[6] + D * q[7];
            double Pn = P * q[0] + D * q[2];
            double Dn = P * q[1] + D * q[3];
            P = Pn;
            D = Dn;
        }
    }
    nb[j] = sp;
    nb[NP.jnear + j] = sm;
}

// ----------------------------------------------------------------- DCT-II --
// chat_n = (eps_n/N) sum_j v_j cos(n theta_j) + dense_n:  DFT of
// p_m = v_{j(m)}, then chat_n = (eps_n/N) Re(e^{i pi n/(2N)} U_n).
// v_j is the sum of the G far-field partials and the near-field value.
__global__ __launch_bounds__(FFT_THREADS) void k_dct2_passA(Geo g, int G, const double* __restrict__ v,
                                                           int64_t v_stride, const double* __restrict__ near,
                                                           int64_t near_stride, int jnear, cplx* __restrict__ X,
                                                           int64_t x_stride) {
    __shared__ cplx buf[FFT_CAP];
    const int N = g.N;
    const int na0 = blockIdx.x * g.colsA;
    const int b = blockIdx.z;
    const double* vb = v + b * v_stride;
    const double* nb = near + b * near_stride;
    const int tot = g.colsA * g.N2;
    for (int e = threadIdx.x; e < tot; e += FFT_THREADS) {
        int col = e % g.colsA, nbi = e / g.colsA;
        int m = na0 + col + g.N1 * nbi;
        int j = row_of(m, N);
        double x = 0;
        for (int q = 0; q < G; ++q) x += vb[(int64_t)q * N + j];
        if (j < jnear) x += nb[j];
        else if (N - 1 - j < jnear) x += nb[jnear + (N - 1 - j)];
        buf[col * g.N2 + nbi] = {x, 0.0};
    }
    __syncthreads();
    lds_fft(buf, g.N2, g.colsA, g.twN2);
    passA_store(g, buf, na0, X + b * x_stride);
}

__global__ __launch_bounds__(FFT_THREADS) void k_dct2_passB(Geo g, int nd, const cplx* __restrict__ X,
                                                           int64_t x_stride, const double* __restrict__ dense,
                                                           int64_t dense_stride, double* __restrict__ chat,
                                                           int64_t chat_stride) {
    __shared__ cplx buf[FFT_CAP];
    const int N = g.N;
    const int jb0 = blockIdx.x * g.rowsB;
    const int b = blockIdx.z;
    passB_load(g, buf, jb0, X + b * x_stride);
    __syncthreads();
    lds_fft(buf, g.N1, g.rowsB, g.twN1);
    const int tot = g.rowsB * g.N1;
    const double* db = dense + b * dense_stride;
    double* cb = chat + b * chat_stride;
    for (int e = threadIdx.x; e < tot; e += FFT_THREADS) {
        int r = e / g.N1, ja = e - r * g.N1;
        int n = jb0 + r + g.N2 * ja;
        cplx U = buf[e];
        cplx t = half_shift(n, N);
        double val = (t.re * U.re - t.im * U.im) * ((n == 0) ? 1.0 : 2.0) / N;
        if (n < nd) val += db[n];
        cb[n] = val;
    }
}

// ------------------------------------------------------------------ NDCT --
// Pair q of Taylor terms (l = 2q: cosine sum of (n/N)^{2q} chat, l = 2q+1:
// sine sum of (n/N)^{2q+1} chat) as one DFT of the Hermitian-split input
//   W_n = (e^{i pi n/(2N)}/2) [x^{2q}(1+x) chat_n - i y^{2q} x chat_{N-n}],
// x = n/N, y = 1 - x (n >= 1), W_0 = chat_0 [q = 0]; then at output m the
// cosine term is Re U_m and the sine term sigma_m Im U_m, row k = j(m).
__global__ __launch_bounds__(FFT_THREADS) void k_ndct_passA(Geo g, int Q, int QG, const double* __restrict__ chat,
                                                           int64_t chat_stride, cplx* __restrict__ X,
                                                           int64_t x_stride) {
    __shared__ cplx buf[FFT_CAP];
    const int N = g.N;
    const int na0 = blockIdx.x * g.colsA;
    const int grp = blockIdx.y;
    const int b = blockIdx.z;
    const double* cb = chat + b * chat_stride;
    cplx* Xb = X + b * x_stride;
    const int tot = g.colsA * g.N2;
    const double invN = 1.0 / N;
    cplx Av[FFT_VPT], Bv[FFT_VPT];
    double px[FFT_VPT], py[FFT_VPT];
    const int q0 = (Q * grp) / QG, q1 = (Q * (grp + 1)) / QG;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        int e = threadIdx.x + s * FFT_THREADS;
        Av[s] = {0, 0};
        Bv[s] = {0, 0};
        px[s] = py[s] = 0;
        if (e < tot) {
            int col = e % g.colsA, nbi = e / g.colsA;
            int n = na0 + col + g.N1 * nbi;
            if (n == 0) {
                Av[s] = {cb[0], 0};
                px[s] = (q0 == 0) ? 1.0 : 0.0;
            } else {
                double x = n * invN, y = (N - n) * invN;
                cplx e2 = cscale(half_shift(n, N), 0.5);
                Av[s] = cscale(e2, (1.0 + x) * cb[n]);
                Bv[s] = cscale(cmuli(e2), -x * cb[N - n]);
                double a = 1, bb = 1;
                for (int q = 0; q < q0; ++q) {
                    a *= x * x;
                    bb *= y * y;
                }
                px[s] = a;
                py[s] = bb;
            }
        }
    }
    for (int q = q0; q < q1; ++q) {
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            int e = threadIdx.x + s * FFT_THREADS;
            if (e < tot) {
                int col = e % g.colsA, nbi = e / g.colsA;
                int n = na0 + col + g.N1 * nbi;
                double x = n * invN, y = (N - n) * invN;
                buf[col * g.N2 + nbi] = cadd(cscale(Av[s], px[s]), cscale(Bv[s], py[s]));
                px[s] *= x * x;
                py[s] *= y * y;
            }
        }
        __syncthreads();
        lds_fft(buf, g.N2, g.colsA, g.twN2);
        passA_store(g, buf, na0, Xb + (int64_t)q * N);
        __syncthreads();
    }
}

// f_k = sum_l s_l d_k^l/l! F_l[k], s_l = (-1)^floor((l+1)/2), d_k = N dtheta_k,
// by Horner from the highest pair down.
__global__ __launch_bounds__(FFT_THREADS) void k_ndct_passB(Geo g, int Q, const cplx* __restrict__ X,
                                                           int64_t x_stride, const double* __restrict__ dth,
                                                           double* __restrict__ f, int64_t f_stride) {
    __shared__ cplx buf[FFT_CAP];
    const int N = g.N;
    const int jb0 = blockIdx.x * g.rowsB;
    const int b = blockIdx.z;
    const cplx* Xb = X + b * x_stride;
    const int tot = g.rowsB * g.N1;
    double acc[FFT_VPT], d[FFT_VPT];
    bool hi[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        int e = threadIdx.x + s * FFT_THREADS;
        acc[s] = 0;
        d[s] = 0;
        hi[s] = false;
        if (e < tot) {
            int r = e / g.N1, ja = e - r * g.N1;
            int m = jb0 + r + g.N2 * ja;
            hi[s] = (2 * m >= N);
            d[s] = (double)N * dth[row_of(m, N)];
        }
    }
    for (int q = Q - 1; q >= 0; --q) {
        passB_load(g, buf, jb0, Xb + (int64_t)q * N);
        __syncthreads();
        lds_fft(buf, g.N1, g.rowsB, g.twN1);
        const double sc = (q & 1) ? -1.0 : 1.0;  // s_{2q} = (-1)^q, s_{2q+1} = -(-1)^q
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            int e = threadIdx.x + s * FFT_THREADS;
            if (e < tot) {
                cplx U = buf[e];
                double Fc = U.re;
                double Fs = hi[s] ? -U.im : U.im;
                double inner = fma(d[s] / (2 * q + 2), acc[s], -sc * Fs);
                acc[s] = fma(d[s] / (2 * q + 1), inner, sc * Fc);
            }
        }
        __syncthreads();
    }
    double* fb = f + b * f_stride;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        int e = threadIdx.x + s * FFT_THREADS;
        if (e < tot) {
            int r = e / g.N1, ja = e - r * g.N1;
            int m = jb0 + r + g.N2 * ja;
            fb[row_of(m, N)] = acc[s];
        }
    }
}


// ============================================================== inverse ===
// c = D_s M^T T^T D_w f (Sec. 4): g = w f; y = T^T g by the transposed Taylor
// series; c_n = (n+1/2) (M^T y)_n with M^T = P^T C D_eps on the grid.

// Transposed Taylor pair q: DFT input at m (row k = j(m)):
//   g_k d_k^{2q} (1 + i sigma_m d_k),  sigma_m = +1 (2m < N), -1 otherwise.
__global__ __launch_bounds__(FFT_THREADS) void k_tndct_passA(Geo g, int Q, int QG, const double* __restrict__ fv,
                                                            int64_t f_stride, const double* __restrict__ wts,
                                                            const double* __restrict__ dth, cplx* __restrict__ X,
                                                            int64_t x_stride) {
    __shared__ cplx buf[FFT_CAP];
    const int N = g.N;
    const int na0 = blockIdx.x * g.colsA;
    const int grp = blockIdx.y;
    const int b = blockIdx.z;
    const double* fb = fv + b * f_stride;
    cplx* Xb = X + b * x_stride;
    const int tot = g.colsA * g.N2;
    double gv[FFT_VPT], dv[FFT_VPT], pw[FFT_VPT];
    const int q0 = (Q * grp) / QG, q1 = (Q * (grp + 1)) / QG;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        int e = threadIdx.x + s * FFT_THREADS;
        gv[s] = dv[s] = pw[s] = 0;
        if (e < tot) {
            int col = e % g.colsA, nbi = e / g.colsA;
            int m = na0 + col + g.N1 * nbi;
            int kk = row_of(m, N);
            gv[s] = wts[kk] * fb[kk];
            dv[s] = (double)N * dth[kk];
            double p = 1;
            for (int q = 0; q < q0; ++q) p *= dv[s] * dv[s];
            pw[s] = p;
        }
    }
    for (int q = q0; q < q1; ++q) {
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            int e = threadIdx.x + s * FFT_THREADS;
            if (e < tot) {
                int col = e % g.colsA, nbi = e / g.colsA;
                int m = na0 + col + g.N1 * nbi;
                double a = gv[s] * pw[s];
                double sg = (2 * m < N) ? 1.0 : -1.0;
                buf[col * g.N2 + nbi] = {a, sg * a * dv[s]};
                pw[s] *= dv[s] * dv[s];
            }
        }
        __syncthreads();
        lds_fft(buf, g.N2, g.colsA, g.twN2);
        passA_store(g, buf, na0, Xb + (int64_t)q * N);
        __syncthreads();
    }
}

// Pass-B tiles closed under n -> N-n: local rows [0, h) are r = tile*h + i
// (r < N2/2) and rows [h, 2h) their partners p(r) = N2 - r (p(0) = N2/2).
__device__ __forceinline__ int pair_row(int tile, int i, int rowsB, int N2) {
    if (N2 == 1) return 0;
    int h = rowsB / 2;
    if (i < h) return tile * h + i;
    int r = tile * h + (i - h);
    return (r == 0) ? N2 / 2 : N2 - r;
}

__device__ __forceinline__ void passB_load_rows(const Geo& g, cplx* buf, int tile, const cplx* __restrict__ X) {
    const int tot = g.rowsB * g.N1;
    for (int e = threadIdx.x; e < tot; e += FFT_THREADS) {
        int i = e % g.rowsB, na = e / g.rowsB;
        buf[i * g.N1 + na] = X[(int64_t)na * g.N2 + pair_row(tile, i, g.rowsB, g.N2)];
    }
}

// y_n = sum_l s_l (n/N)^l / l! Z_l[n]; Z_{2q} = Re(e_n A_n), Z_{2q+1} = Im(e_n B_n),
// A = (U_n + conj U_{N-n})/2, B = (U_n - conj U_{N-n})/(2i), e_n = e^{i pi n/(2N)}.
__global__ __launch_bounds__(FFT_THREADS) void k_tndct_passB(Geo g, int Q, const cplx* __restrict__ X,
                                                            int64_t x_stride, double* __restrict__ y,
                                                            int64_t y_stride) {
    __shared__ cplx buf[FFT_CAP];
    const int N = g.N;
    const int tile = blockIdx.x;
    const int b = blockIdx.z;
    const cplx* Xb = X + b * x_stride;
    const int tot = g.rowsB * g.N1;
    const int nrows = (g.N2 == 1) ? 1 : g.rowsB;
    const int h = g.rowsB / 2;
    double acc[FFT_VPT], xs[FFT_VPT];
    cplx en[FFT_VPT];
    int part[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        int e = threadIdx.x + s * FFT_THREADS;
        acc[s] = 0;
        xs[s] = 0;
        en[s] = {0, 0};
        part[s] = 0;
        if (e < tot && e / g.N1 < nrows) {
            int i = e / g.N1, ja = e - i * g.N1;
            int r = pair_row(tile, i, g.rowsB, g.N2);
            int n = r + g.N2 * ja;
            xs[s] = (double)n / N;
            en[s] = half_shift(n, N);
            int ip, jp;
            if (r == 0) {
                ip = i;
                jp = (g.N1 - ja) & (g.N1 - 1);
            } else {
                ip = (g.N2 == 1) ? i : (i < h ? i + h : i - h);
                if (r == g.N2 / 2) ip = i;
                jp = g.N1 - 1 - ja;
            }
            part[s] = ip * g.N1 + jp;
        }
    }
    for (int q = Q - 1; q >= 0; --q) {
        passB_load_rows(g, buf, tile, Xb + (int64_t)q * N);
        __syncthreads();
        lds_fft(buf, g.N1, g.rowsB, g.twN1);
        const double sc = (q & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) {
            int e = threadIdx.x + s * FFT_THREADS;
            if (e < tot && e / g.N1 < nrows) {
                cplx U = buf[e], V = buf[part[s]];
                cplx A = {0.5 * (U.re + V.re), 0.5 * (U.im - V.im)};
                cplx Bm = {0.5 * (U.im + V.im), -0.5 * (U.re - V.re)};  // (U - conj V)/(2i)
                double Zc = en[s].re * A.re - en[s].im * A.im;
                double Zs = en[s].re * Bm.im + en[s].im * Bm.re;
                double inner = fma(xs[s] / (2 * q + 2), acc[s], -sc * Zs);
                acc[s] = fma(xs[s] / (2 * q + 1), inner, sc * Zc);
            }
        }
        __syncthreads();
    }
    double* yb = y + b * y_stride;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        int e = threadIdx.x + s * FFT_THREADS;
        if (e < tot && e / g.N1 < nrows) {
            int i = e / g.N1, ja = e - i * g.N1;
            int r = pair_row(tile, i, g.rowsB, g.N2);
            yb[r + g.N2 * ja] = acc[s];
        }
    }
}

// (M^T y)_n for n < nd, chunk blockIdx.y of rows k:
//   sum_{k in chunk, k <= n, k+n even} (eps_k/pi) Lam((n-k)/2) Lam((n+k)/2) y_k
__global__ void k_dense_t(int nd, int chunk, const double* __restrict__ lam, const double* __restrict__ y,
                          int64_t y_stride, double* __restrict__ part, int64_t part_stride) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    int ch = blockIdx.y;
    int b = blockIdx.z;
    if (n >= nd) return;
    const double* yb = y + b * y_stride;
    int k0 = ch * chunk, k1 = min(n + 1, k0 + chunk);
    int k = k0;
    if ((n - k) & 1) ++k;
    double acc = 0;
    for (; k < k1; k += 2) {
        double e = (k == 0) ? 0.3183098861837907 : 0.6366197723675814;
        acc = fma(e * lam[(n - k) >> 1] * lam[(n + k) >> 1], yb[k], acc);
    }
    part[b * part_stride + (int64_t)ch * nd + n] = acc;
}

__global__ void k_dense_t_reduce(int nd, int nchunk, int chunk, const double* __restrict__ part,
                                 int64_t part_stride, double* __restrict__ out, int64_t out_stride) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.z;
    if (n >= nd) return;
    const double* pb = part + b * part_stride;
    double s = 0;
    int last = min(nchunk - 1, n / chunk);
    for (int ch = 0; ch <= last; ++ch) s += pb[(int64_t)ch * nd + n];
    out[b * out_stride + n] = s;
}

// u_j = sum_k (eps_k/N) y_k cos(k theta_j): DFT of (eps_k/N) y_k e^{i pi k/(2N)},
// u at row j(m) = Re V_m.
__global__ __launch_bounds__(FFT_THREADS) void k_dct3_passA(Geo g, const double* __restrict__ y, int64_t y_stride,
                                                           cplx* __restrict__ X, int64_t x_stride) {
    __shared__ cplx buf[FFT_CAP];
    const int N = g.N;
    const int na0 = blockIdx.x * g.colsA;
    const int b = blockIdx.z;
    const double* yb = y + b * y_stride;
    const int tot = g.colsA * g.N2;
    for (int e = threadIdx.x; e < tot; e += FFT_THREADS) {
        int col = e % g.colsA, nbi = e / g.colsA;
        int n = na0 + col + g.N1 * nbi;
        double a = yb[n] * ((n == 0) ? 1.0 : 2.0) / N;
        buf[col * g.N2 + nbi] = cscale(half_shift(n, N), a);
    }
    __syncthreads();
    lds_fft(buf, g.N2, g.colsA, g.twN2);
    passA_store(g, buf, na0, X + b * x_stride);
}

__global__ __launch_bounds__(FFT_THREADS) void k_dct3_passB(Geo g, const cplx* __restrict__ X, int64_t x_stride,
                                                           double* __restrict__ u, int64_t u_stride) {
    __shared__ cplx buf[FFT_CAP];
    const int N = g.N;
    const int jb0 = blockIdx.x * g.rowsB;
    const int b = blockIdx.z;
    passB_load(g, buf, jb0, X + b * x_stride);
    __syncthreads();
    lds_fft(buf, g.N1, g.rowsB, g.twN1);
    const int tot = g.rowsB * g.N1;
    double* ub = u + b * u_stride;
    for (int e = threadIdx.x; e < tot; e += FFT_THREADS) {
        int r = e / g.N1, ja = e - r * g.N1;
        int m = jb0 + r + g.N2 * ja;
        ub[row_of(m, N)] = buf[e].re;
    }
}

// Transposed far field, pass A: for every term (b, m), ascending m, the DFT
// input at m is rho at row j = j(m) (conjugated when 2m >= N) with
//   rho_j = u_j e^{i (m+1/2)(theta_j - pi/2)} (2 sin theta_j)^{-m-1/2} [j in block b].
__global__ __launch_bounds__(FFT_THREADS) void k_tfar_passA(Geo g, FarParams F, const double* __restrict__ u,
                                                           int64_t u_stride, cplx* __restrict__ X,
                                                           int64_t x_stride) {
    __shared__ cplx buf[FFT_CAP];
    const int N = g.N;
    const int na0 = blockIdx.x * g.colsA;
    const int b = blockIdx.z;
    const double* ub = u + b * u_stride;
    cplx* Xb = X + b * x_stride;
    const int tot = g.colsA * g.N2;
    const double pi = 3.141592653589793;
    cplx gm[FFT_VPT], rq[FFT_VPT];
    int blk[FFT_VPT];
    bool cj[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        int e = threadIdx.x + s * FFT_THREADS;
        gm[s] = rq[s] = {0, 0};
        blk[s] = -1;
        cj[s] = false;
        if (e < tot) {
            int col = e % g.colsA, nbi = e / g.colsA;
            int m = na0 + col + g.N1 * nbi;
            int j = row_of(m, N);
            cj[s] = (2 * m >= N);
            blk[s] = row_block(F, j, N);
            double d = pi * (double)(2 * j + 1 - N) / (2.0 * N);
            int jj = min(j, N - 1 - j);
            double sn = sin((jj + 0.5) * pi / N);
            double q = 1.0 / (2.0 * sn);
            double ps, pc, rs, rc;
            sincos(0.5 * d, &ps, &pc);
            sincos(d, &rs, &rc);
            double r0 = sqrt(q) * ub[j];
            gm[s] = {pc * r0, ps * r0};
            rq[s] = {rc * q, rs * q};
        }
    }
    for (int m = 0; m < F.Mmax; ++m) {
        for (int t = 0; t < F.nterm; ++t) {
            if (F.term_m[t] != m) continue;
            const int tb = F.term_blk[t];
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) {
                int e = threadIdx.x + s * FFT_THREADS;
                if (e < tot) {
                    int col = e % g.colsA, nbi = e / g.colsA;
                    cplx v = (blk[s] == tb) ? gm[s] : cplx{0, 0};
                    if (cj[s]) v.im = -v.im;
                    buf[col * g.N2 + nbi] = v;
                }
            }
            __syncthreads();
            lds_fft(buf, g.N2, g.colsA, g.twN2);
            passA_store(g, buf, na0, Xb + (int64_t)t * N);
            __syncthreads();
        }
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s) gm[s] = cmul(gm[s], rq[s]);
    }
}

// Transposed far field, pass B: out_n = sum_terms C_n h_{m,n} [n >= nlo_b]
// Re(e^{i pi n/(2N)} U_n), descending m (h by multiplication only).
__global__ __launch_bounds__(FFT_THREADS) void k_tfar_passB(Geo g, FarParams F, const cplx* __restrict__ X,
                                                           int64_t x_stride, double* __restrict__ out,
                                                           int64_t out_stride) {
    __shared__ cplx buf[FFT_CAP];
    const int N = g.N;
    const int jb0 = blockIdx.x * g.rowsB;
    const int b = blockIdx.z;
    const cplx* Xb = X + b * x_stride;
    const int tot = g.rowsB * g.N1;
    double acc[FFT_VPT], h[FFT_VPT];
    cplx en[FFT_VPT];
    int nn[FFT_VPT];
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        int e = threadIdx.x + s * FFT_THREADS;
        acc[s] = 0;
        h[s] = 0;
        en[s] = {0, 0};
        nn[s] = -1;
        if (e < tot) {
            int r = e / g.N1, ja = e - r * g.N1;
            int n = jb0 + r + g.N2 * ja;
            nn[s] = n;
            if (n >= F.nd) {
                en[s] = cscale(half_shift(n, N), stieltjes_C((double)n));
                double hv = 1;
                for (int j = 1; j < F.Mmax; ++j) hv *= (j - 0.5) * (j - 0.5) / (j * (n + j + 0.5));
                h[s] = hv;
            }
        }
    }
    for (int m = F.Mmax - 1; m >= 0; --m) {
        for (int t = 0; t < F.nterm; ++t) {
            if (F.term_m[t] != m) continue;
            const int nlo = F.blk[F.term_blk[t]].nlo;
            passB_load(g, buf, jb0, Xb + (int64_t)t * N);
            __syncthreads();
            lds_fft(buf, g.N1, g.rowsB, g.twN1);
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s) {
                int e = threadIdx.x + s * FFT_THREADS;
                if (e < tot && nn[s] >= nlo) {
                    cplx U = buf[e];
                    acc[s] = fma(h[s], en[s].re * U.re - en[s].im * U.im, acc[s]);
                }
            }
            __syncthreads();
        }
        if (m > 0) {
#pragma unroll
            for (int s = 0; s < FFT_VPT; ++s)
                if (nn[s] >= 0) h[s] *= m * (nn[s] + m + 0.5) / ((m - 0.5) * (m - 0.5));
        }
    }
    double* ob = out + b * out_stride;
#pragma unroll
    for (int s = 0; s < FFT_VPT; ++s) {
        int e = threadIdx.x + s * FFT_THREADS;
        if (e < tot) ob[nn[s]] = acc[s];
    }
}

// Transposed near field.  (1) k_near_items with c == null gives each
// (row, chunk) transfer matrix; (2) k_tnear_scan chains them per row into the
// state (P, D) at every chunk start; (3) k_tnear_accum reruns each chunk from
// its true state for 256 rows of one segment and sums over the rows
//   out_n += P_n(x_j) (u_j + (-1)^n u_{N-1-j})
// through an LDS tile, 32 degrees at a time.
__global__ void k_tnear_scan(NearParams NP, const double* __restrict__ items, int64_t it_stride,
                             double* __restrict__ st, int64_t st_stride) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.z;
    if (j >= NP.jnear) return;
    int sgi = -1;
    for (int s = 0; s < NP.nseg; ++s)
        if (j >= NP.seg[s].jlo && j < NP.seg[s].jhi) sgi = s;
    if (sgi < 0) return;
    const Seg S = NP.seg[sgi];
    const double* it = items + b * it_stride;
    double* so = st + b * st_stride;
    int nrows = S.jhi - S.jlo;
    double P = 1, D = 0;
    for (int ch = 0; ch < S.nchunk; ++ch) {
        int id = S.item_off + ch * nrows + (j - S.jlo);
        so[2 * id] = P;
        so[2 * id + 1] = D;
        const double* q = it + (int64_t)id * 8;
        if (ch == 0) {
            P = q[0];
            D = q[1];
        } else {
            double Pn = P * q[0] + D * q[2];
            double Dn = P * q[1] + D * q[3];
            P = Pn;
            D = Dn;
        }
    }
}

constexpr int TN_ROWS = 256;
constexpr int TN_STEPS = 32;

// grid.x enumerates (segment, chunk, row group) with the table from the plan
__global__ __launch_bounds__(TN_ROWS) void k_tnear_accum(int N, NearParams NP, const int* __restrict__ wg_seg,
                                                          const int* __restrict__ wg_rg_off,
                                                          const double* __restrict__ A,
                                                          const double* __restrict__ B, const double* __restrict__ u,
                                                          int64_t u_stride, const double* __restrict__ st,
                                                          int64_t st_stride, double* __restrict__ part,
                                                          int64_t part_stride) {
    __shared__ double tile[TN_STEPS][TN_ROWS + 1];
    const int wgid = blockIdx.x;
    const int b = blockIdx.z;
    const int sgi = wg_seg[wgid];
    const Seg S = NP.seg[sgi];
    const int nrows = S.jhi - S.jlo;
    const int ngroups = (nrows + TN_ROWS - 1) / TN_ROWS;
    // local index inside the segment: chunk-major over row groups
    int loc = wgid - wg_rg_off[2 * sgi];
    int ch = loc / ngroups;
    int grp = loc - ch * ngroups;
    int rg_global = wg_rg_off[2 * sgi + 1] + grp;
    int row = grp * TN_ROWS + threadIdx.x;
    bool act = row < nrows;
    int j = S.jlo + (act ? row : 0);
    const double* ub = u + b * u_stride;
    const double* so = st + b * st_stride;
    double uj = act ? ub[j] : 0.0, um = act ? ub[N - 1 - j] : 0.0;
    const double pi = 3.141592653589793;
    double sn = sin(0.5 * (j + 0.5) * pi / N);
    double uu = 2.0 * sn * sn;
    int id = S.item_off + ch * nrows + (act ? row : 0);
    double p = act ? so[2 * id] : 0.0, d = act ? so[2 * id + 1] : 0.0;
    int n0 = ch * NEAR_CHUNK, n1 = min(S.nend, n0 + NEAR_CHUNK);
    double* pb = part + b * part_stride + (int64_t)rg_global * N;
    for (int nb0 = n0; nb0 < n1; nb0 += TN_STEPS) {
        int cnt = min(TN_STEPS, n1 - nb0);
        for (int i = 0; i < cnt; ++i) {
            int n = nb0 + i;
            tile[i][threadIdx.x] = p * ((n & 1) ? uj - um : uj + um);
            double dn = fma(A[n], d, -B[n] * uu * p);
            p += dn;
            d = dn;
        }
        __syncthreads();
        // 8 threads per degree column, 32 rows each, then a butterfly of 8
        int col = threadIdx.x >> 3, prt = threadIdx.x & 7;
        double s = 0;
        if (col < cnt)
            for (int r = 0; r < TN_ROWS / 8; ++r) s += tile[col][prt * (TN_ROWS / 8) + r];
        s += __shfl_xor(s, 1, 8);
        s += __shfl_xor(s, 2, 8);
        s += __shfl_xor(s, 4, 8);
        if (prt == 0 && col < cnt) pb[nb0 + col] = s;
        __syncthreads();
    }
}

// c_n = (n + 1/2) (dense_n [n < nd] + far_n + sum_rg near parts [nd <= n < nend(rg)])
__global__ void k_idlt_final(int N, int nd, int nrg, const int* __restrict__ rg_nend, const double* __restrict__ dense,
                             int64_t dense_stride, const double* __restrict__ far, int64_t far_stride,
                             const double* __restrict__ part, int64_t part_stride, double* __restrict__ c,
                             int64_t c_stride) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.z;
    if (n >= N) return;
    double s;
    if (n < nd) {
        s = dense[b * dense_stride + n];
    } else {
        s = far ? far[b * far_stride + n] : 0.0;
        const double* pb = part + b * part_stride;
        for (int r = 0; r < nrg; ++r)
            if (n < rg_nend[r]) s += pb[(int64_t)r * N + n];
    }
    c[b * c_stride + n] = (n + 0.5) * s;
}

}  // namespace dlt

// ================================================================ host ====
namespace dlt {

// ---- kernel trace: start/stop events around every launch while enabled
namespace trace {
struct Rec {
    const char* name;
    hipEvent_t a, b;
};
static std::mutex mu;
static bool on = false;
static std::vector<Rec> recs;
static std::vector<hipEvent_t> pool;

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

void trace_set(bool enable) {
    std::lock_guard<std::mutex> lk(trace::mu);
    trace::on = enable;
}

// launches `fn` bracketed by events when tracing
template <class F>
static void traced(const char* name, hipStream_t s, F&& fn) {
    if (!trace::on) {
        fn();
        return;
    }
    std::lock_guard<std::mutex> lk(trace::mu);
    trace::Rec r{name, trace::take(), trace::take()};
    (void)hipEventRecord(r.a, s);
    fn();
    (void)hipEventRecord(r.b, s);
    trace::recs.push_back(r);
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
    w.states = (double*)take(p.ws_states);
    w.sstates = (int64_t)(al256(p.ws_states) / sizeof(double));
    w.part = (double*)take(p.ws_part);
    w.spart = (int64_t)(al256(p.ws_part) / sizeof(double));
}

hipError_t run_nodes(const Plan& p, double* theta, double* w, double* dth, hipStream_t s) {
    const NodeParams& P = p.nodes;
    int nh = (P.N + 1) / 2;
    if (P.kb > 0) {
        size_t shm = (7 * 256 + 3) * sizeof(double);
        traced("k_nodes_boundary", s, [&] { k_nodes_boundary<<<P.kb, 256, shm, s>>>(P, p.d_guess, p.d_recA, p.d_recB, theta, w, dth); });
    }
    int ni = nh - P.kb;
    if (ni > 0)
        traced("k_nodes_interior", s, [&] { k_nodes_interior<<<(ni + 255) / 256, 256, 0, s>>>(P, theta, w, dth); });
    return hipGetLastError();
}

hipError_t run_leg2cheb(const Plan& p, int64_t nb, const double* c, double* chat, Work& w, hipStream_t s) {
    const int N = (int)p.N;
    const int nd = p.nd;
    const Geo& g = p.geo;
    // dense block: partials then reduction into the last slab of `dense`
    double* dense_out = w.dense + (int64_t)p.dense_nchunk * nd;
    dim3 gd((nd + 255) / 256, p.dense_nchunk, (unsigned)nb);
    traced("k_dense", s, [&] { k_dense<<<gd, 256, 0, s>>>(N, nd, p.dense_chunk, p.d_lam, c, N, w.dense, w.sdense); });
    if (N <= nd) {
        traced("k_dense_reduce", s, [&] { k_dense_reduce<<<dim3((nd + 255) / 256, 1, (unsigned)nb), 256, 0, s>>>(nd, p.dense_nchunk, p.dense_chunk,
                                                                           w.dense, w.sdense, chat, N); });
        return hipGetLastError();
    }
    traced("k_dense_reduce", s, [&] { k_dense_reduce<<<dim3((nd + 255) / 256, 1, (unsigned)nb), 256, 0, s>>>(nd, p.dense_nchunk, p.dense_chunk,
                                                                       w.dense, w.sdense, dense_out, w.sdense); });
    // near field
    const NearParams& NP = p.near;
    if (NP.nitems > 0)
        traced("k_near_items", s, [&] { k_near_items<<<dim3((NP.nitems + 255) / 256, 1, (unsigned)nb), 256, 0, s>>>(N, NP, p.d_recA, p.d_recB, c, N,
                                                                                w.items, w.sitems); });
    if (NP.jnear > 0)
        traced("k_near_combine", s, [&] { k_near_combine<<<dim3((NP.jnear + 255) / 256, 1, (unsigned)nb), 256, 0, s>>>(NP, w.items, w.sitems, w.near,
                                                                                 w.snear); });
    // far field
    const FarParams& F = p.far;
    traced("k_far_passA", s, [&] { k_far_passA<<<dim3(g.N1 / g.colsA, 1, (unsigned)nb), FFT_THREADS, 0, s>>>(g, F, c, N, w.X, w.sX); });
    traced("k_far_passB", s, [&] { k_far_passB<<<dim3(g.N2 / g.rowsB, p.tgB, (unsigned)nb), FFT_THREADS, 0, s>>>(g, F, p.tgB, w.X, w.sX, w.v,
                                                                               w.sv); });
    // values on the grid -> coefficients
    traced("k_dct2_passA", s, [&] { k_dct2_passA<<<dim3(g.N1 / g.colsA, 1, (unsigned)nb), FFT_THREADS, 0, s>>>(g, p.tgB, w.v, w.sv, w.near, w.snear,
                                                                            NP.jnear, w.X, w.sX); });
    traced("k_dct2_passB", s, [&] { k_dct2_passB<<<dim3(g.N2 / g.rowsB, 1, (unsigned)nb), FFT_THREADS, 0, s>>>(g, nd, w.X, w.sX, dense_out, w.sdense,
                                                                            chat, N); });
    return hipGetLastError();
}

hipError_t run_ndct(const Plan& p, int64_t nb, const double* chat, const double* dth, double* f, Work& w,
                    hipStream_t s) {
    const Geo& g = p.geo;
    const int Q = p.L / 2;
    const int tilesA = g.N1 / g.colsA;
    // small transforms: split the Taylor pairs over blocks for parallelism
    int QG = (tilesA * nb >= 256) ? 1 : Q;
    traced("k_ndct_passA", s, [&] { k_ndct_passA<<<dim3(tilesA, QG, (unsigned)nb), FFT_THREADS, 0, s>>>(g, Q, QG, chat, p.N, w.X, w.sX); });
    traced("k_ndct_passB", s, [&] { k_ndct_passB<<<dim3(g.N2 / g.rowsB, 1, (unsigned)nb), FFT_THREADS, 0, s>>>(g, Q, w.X, w.sX, dth, f, p.N); });
    return hipGetLastError();
}

hipError_t run_inverse(const Plan& p, int64_t nb, const double* f, const double* wts, const double* dth,
                       double* c, Work& w, hipStream_t s) {
    const int N = (int)p.N;
    const int nd = p.nd;
    const Geo& g = p.geo;
    const int Q = p.L / 2;
    const int tilesA = g.N1 / g.colsA;
    int QG = (tilesA * nb >= 256) ? 1 : Q;
    double* y = w.chat;  // T^T D_w f, stride w.schat
    // transposed Taylor series: y = T^T (w f)
    traced("k_tndct_passA", s, [&] { k_tndct_passA<<<dim3(tilesA, QG, (unsigned)nb), FFT_THREADS, 0, s>>>(g, Q, QG, f, N, wts, dth, w.X, w.sX); });
    int tilesB = (g.N2 == 1) ? 1 : g.N2 / g.rowsB;
    traced("k_tndct_passB", s, [&] { k_tndct_passB<<<dim3(tilesB, 1, (unsigned)nb), FFT_THREADS, 0, s>>>(g, Q, w.X, w.sX, y, w.schat); });
    // dense block of M^T for n < nd
    double* dense_out = w.dense + (int64_t)p.dense_nchunk * nd;
    traced("k_dense_t", s, [&] { k_dense_t<<<dim3((nd + 255) / 256, p.dense_nchunk, (unsigned)nb), 256, 0, s>>>(nd, p.dense_chunk, p.d_lam, y,
                                                                                 w.schat, w.dense, w.sdense); });
    traced("k_dense_t_reduce", s, [&] { k_dense_t_reduce<<<dim3((nd + 255) / 256, 1, (unsigned)nb), 256, 0, s>>>(nd, p.dense_nchunk, p.dense_chunk,
                                                                         w.dense, w.sdense, dense_out, w.sdense); });
    const double* far = nullptr;
    const NearParams& NP = p.near;
    if (N > nd) {
        // u = C D_eps y on the grid
        double* u = w.vec;
        traced("k_dct3_passA", s, [&] { k_dct3_passA<<<dim3(tilesA, 1, (unsigned)nb), FFT_THREADS, 0, s>>>(g, y, w.schat, w.X, w.sX); });
        traced("k_dct3_passB", s, [&] { k_dct3_passB<<<dim3(g.N2 / g.rowsB, 1, (unsigned)nb), FFT_THREADS, 0, s>>>(g, w.X, w.sX, u, w.svec); });
        // transposed far field
        traced("k_tfar_passA", s, [&] { k_tfar_passA<<<dim3(tilesA, 1, (unsigned)nb), FFT_THREADS, 0, s>>>(g, p.far, u, w.svec, w.X, w.sX); });
        traced("k_tfar_passB", s, [&] { k_tfar_passB<<<dim3(g.N2 / g.rowsB, 1, (unsigned)nb), FFT_THREADS, 0, s>>>(g, p.far, w.X, w.sX, w.v, w.sv); });
        far = w.v;
        // transposed near field
        if (NP.nitems > 0) {
            traced("k_near_items", s, [&] { k_near_items<<<dim3((NP.nitems + 255) / 256, 1, (unsigned)nb), 256, 0, s>>>(
                N, NP, p.d_recA, p.d_recB, nullptr, 0, w.items, w.sitems); });
            traced("k_tnear_scan", s, [&] { k_tnear_scan<<<dim3((NP.jnear + 255) / 256, 1, (unsigned)nb), 256, 0, s>>>(NP, w.items, w.sitems,
                                                                                    w.states, w.sstates); });
            traced("k_tnear_accum", s, [&] { k_tnear_accum<<<dim3(p.tn_wg, 1, (unsigned)nb), TN_ROWS, 0, s>>>(
                N, NP, p.d_tn_wgseg, p.d_tn_segoff, p.d_recA, p.d_recB, u, w.svec, w.states, w.sstates, w.part,
                w.spart); });
        }
    }
    traced("k_idlt_final", s, [&] { k_idlt_final<<<dim3((N + 255) / 256, 1, (unsigned)nb), 256, 0, s>>>(
        N, nd, (N > nd) ? p.tn_nrg : 0, p.d_tn_rgnend, dense_out, w.sdense, far, w.sv, w.part, w.spart, c, N); });
    return hipGetLastError();
}

}  // namespace dlt
