// Device-side building blocks shared by the DLT kernels: complex arithmetic,
// twiddle access, the LDS-resident FFT, and the Gamma-ratio series used by
// the asymptotic (Stieltjes) expansion of P_n(cos theta).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dlt {

struct cplx {
    double re, im;
};

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ cplx cconj(cplx a) { return {a.re, -a.im}; }
// multiply by +i
__device__ __forceinline__ cplx cmuli(cplx a) { return {-a.im, a.re}; }

// Threads per block of every FFT-carrying kernel, and the LDS capacity in
// complex doubles one block uses for its tile (32 KiB).
constexpr int FFT_THREADS = 256;
constexpr int FFT_CAP = 2048;
constexpr int FFT_VPT = FFT_CAP / FFT_THREADS;  // values per thread per stage
// LDS tiles are padded with one complex per 8 so that the stride-4 writes of
// the first Stockham stage fall into distinct banks
constexpr int FFT_LDS = FFT_CAP + FFT_CAP / 8;
__device__ __forceinline__ int lp(int x) { return x + (x >> 3); }

// e^{+2 pi i t / len} from a table tw[t] = e^{+2 pi i t / len}, t < len.
__device__ __forceinline__ cplx tw_load(const cplx* __restrict__ tw, int t) { return tw[t]; }

// e^{+2 pi i t / N}, 0 <= t < N, from a two-level table:
//   hi[t >> sh] = e^{2 pi i (t >> sh) 2^sh / N},  lo[t & mask] = e^{2 pi i (t & mask)/N}.
__device__ __forceinline__ cplx tw2(const cplx* __restrict__ hi, const cplx* __restrict__ lo, int64_t t,
                                    int sh) {
    cplx a = hi[t >> sh];
    cplx b = lo[t & ((int64_t(1) << sh) - 1)];
    return cmul(a, b);
}

// In-place radix-4 (one radix-2 stage when log2(len) is odd) Stockham FFT with
// the + sign, sum_n x_n e^{+2 pi i n m/len}, of `cols` independent sequences
// stored contiguously in LDS: buf[lp(col*len + i)], cols*len <= FFT_CAP.  Every
// thread of the (FFT_THREADS-wide) block must call it.  `tw` is the table of
// e^{+2 pi i t/len}.  Each stage reads all of its inputs into registers, waits,
// then writes, so one buffer suffices.
__device__ inline void lds_fft(cplx* buf, int len, int cols, const cplx* __restrict__ tw) {
    const int tid = threadIdx.x;
    for (int p = 1; p < len;) {
        const int r = ((len / p) & 3) == 0 ? 4 : 2;
        const int nb = len / r;
        const int total = nb * cols;
        const int tstride = len / (p * r);
        cplx v[FFT_VPT];
        int dst[FFT_VPT / 2];
        if (r == 4) {
#pragma unroll
            for (int b = 0; b < FFT_VPT / 4; ++b) {
                int t = tid + b * FFT_THREADS;
                if (t < total) {
                    int col = t / nb;
                    int i = t - col * nb;
                    int k = i & (p - 1);
                    const int cb0 = col * len;
                    cplx x0 = buf[lp(cb0 + i)], x1 = buf[lp(cb0 + i + nb)], x2 = buf[lp(cb0 + i + 2 * nb)], x3 = buf[lp(cb0 + i + 3 * nb)];
                    if (p > 1) {
                        cplx w1 = tw_load(tw, k * tstride);
                        cplx w2 = cmul(w1, w1);
                        cplx w3 = cmul(w2, w1);
                        x1 = cmul(x1, w1);
                        x2 = cmul(x2, w2);
                        x3 = cmul(x3, w3);
                    }
                    cplx s02 = cadd(x0, x2), d02 = csub(x0, x2);
                    cplx s13 = cadd(x1, x3), d13 = cmuli(csub(x1, x3));
                    v[4 * b + 0] = cadd(s02, s13);
                    v[4 * b + 1] = cadd(d02, d13);
                    v[4 * b + 2] = csub(s02, s13);
                    v[4 * b + 3] = csub(d02, d13);
                    dst[b] = col * len + (i - k) * 4 + k;
                }
            }
            __syncthreads();
#pragma unroll
            for (int b = 0; b < FFT_VPT / 4; ++b) {
                int t = tid + b * FFT_THREADS;
                if (t < total) {
                    int d = dst[b];
                    buf[lp(d)] = v[4 * b + 0];
                    buf[lp(d + p)] = v[4 * b + 1];
                    buf[lp(d + 2 * p)] = v[4 * b + 2];
                    buf[lp(d + 3 * p)] = v[4 * b + 3];
                }
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int b = 0; b < FFT_VPT / 2; ++b) {
                int t = tid + b * FFT_THREADS;
                if (t < total) {
                    int col = t / nb;
                    int i = t - col * nb;
                    int k = i & (p - 1);
                    const int cb0 = col * len;
                    cplx x0 = buf[lp(cb0 + i)], x1 = buf[lp(cb0 + i + nb)];
                    if (p > 1) x1 = cmul(x1, tw_load(tw, k * tstride));
                    v[2 * b + 0] = cadd(x0, x1);
                    v[2 * b + 1] = csub(x0, x1);
                    dst[b] = col * len + (i - k) * 2 + k;
                }
            }
            __syncthreads();
#pragma unroll
            for (int b = 0; b < FFT_VPT / 2; ++b) {
                int t = tid + b * FFT_THREADS;
                if (t < total) {
                    int d = dst[b];
                    buf[lp(d)] = v[2 * b + 0];
                    buf[lp(d + p)] = v[2 * b + 1];
                }
            }
            __syncthreads();
        }
        p *= r;
    }
}

// Same transform with the length known at compile time (L > 0) so that the
// stage loop unrolls and index arithmetic becomes shifts; L == 0 falls back
// to the run-time length `len`.
template <int L>
__device__ __forceinline__ void lds_fft_t(cplx* buf, int len, int cols, const cplx* __restrict__ tw) {
    if constexpr (L == 0) {
        lds_fft(buf, len, cols, tw);
    } else {
        constexpr int LOG = __builtin_ctz(L);
        const int tid = threadIdx.x;
#pragma unroll
        for (int st = 0; st < (LOG + 1) / 2; ++st) {
            // radix 4 while two or more bits remain, radix 2 for a last odd bit
            const int p = 1 << (2 * st);
            const int r = ((LOG - 2 * st) >= 2) ? 4 : 2;
            const int nb = L / r;
            const int total = nb * cols;
            const int tstride = L / (p * r);
            cplx v[FFT_VPT];
            int dst[FFT_VPT / 2];
            if (r == 4) {
#pragma unroll
                for (int b = 0; b < FFT_VPT / 4; ++b) {
                    int t = tid + b * FFT_THREADS;
                    if (t < total) {
                        int col = t / nb;
                        int i = t - col * nb;
                        int k = i & (p - 1);
                        const int cb0 = col * L;
                        cplx x0 = buf[lp(cb0 + i)], x1 = buf[lp(cb0 + i + nb)], x2 = buf[lp(cb0 + i + 2 * nb)], x3 = buf[lp(cb0 + i + 3 * nb)];
                        if (p > 1) {
                            cplx w1 = tw[k * tstride];
                            cplx w2 = cmul(w1, w1);
                            cplx w3 = cmul(w2, w1);
                            x1 = cmul(x1, w1);
                            x2 = cmul(x2, w2);
                            x3 = cmul(x3, w3);
                        }
                        cplx s02 = cadd(x0, x2), d02 = csub(x0, x2);
                        cplx s13 = cadd(x1, x3), d13 = cmuli(csub(x1, x3));
                        v[4 * b + 0] = cadd(s02, s13);
                        v[4 * b + 1] = cadd(d02, d13);
                        v[4 * b + 2] = csub(s02, s13);
                        v[4 * b + 3] = csub(d02, d13);
                        dst[b] = col * L + (i - k) * 4 + k;
                    }
                }
                __syncthreads();
#pragma unroll
                for (int b = 0; b < FFT_VPT / 4; ++b) {
                    int t = tid + b * FFT_THREADS;
                    if (t < total) {
                        int d = dst[b];
                        buf[lp(d)] = v[4 * b + 0];
                        buf[lp(d + p)] = v[4 * b + 1];
                        buf[lp(d + 2 * p)] = v[4 * b + 2];
                        buf[lp(d + 3 * p)] = v[4 * b + 3];
                    }
                }
                __syncthreads();
            } else {
#pragma unroll
                for (int b = 0; b < FFT_VPT / 2; ++b) {
                    int t = tid + b * FFT_THREADS;
                    if (t < total) {
                        int col = t / nb;
                        int i = t - col * nb;
                        int k = i & (p - 1);
                        const int cb0 = col * L;
                        cplx x0 = buf[lp(cb0 + i)], x1 = buf[lp(cb0 + i + nb)];
                        if (p > 1) x1 = cmul(x1, tw[k * tstride]);
                        v[2 * b + 0] = cadd(x0, x1);
                        v[2 * b + 1] = csub(x0, x1);
                        dst[b] = col * L + (i - k) * 2 + k;
                    }
                }
                __syncthreads();
#pragma unroll
                for (int b = 0; b < FFT_VPT / 2; ++b) {
                    int t = tid + b * FFT_THREADS;
                    if (t < total) {
                        int d = dst[b];
                        buf[lp(d)] = v[2 * b + 0];
                        buf[lp(d + p)] = v[2 * b + 1];
                    }
                }
                __syncthreads();
            }
        }
    }
}

// Gamma(x+1/2)/Gamma(x) for x >= 10 from its Stirling-type expansion
//   log(Gamma(x+1/2)/Gamma(x)) = log(x)/2 + sum_k a_k / x^(2k-1),
//   a_k = B_{2k} (2^{1-2k} - 2) / ((2k-1) 2k)  (B_j Bernoulli numbers),
// eight terms: relative error below 1e-17 for x >= 10.
__device__ __forceinline__ double gamma_half_ratio_series(double x) {
    const double r = 1.0 / x;
    const double r2 = r * r;
    double s = 929569.0 / 15728640.0;
    s = fma(s, r2, -5461.0 / 425984.0);
    s = fma(s, r2, 691.0 / 180224.0);
    s = fma(s, r2, -31.0 / 18432.0);
    s = fma(s, r2, 17.0 / 14336.0);
    s = fma(s, r2, -1.0 / 640.0);
    s = fma(s, r2, 1.0 / 192.0);
    s = fma(s, r2, -1.0 / 8.0);
    s *= r;
    return sqrt(x) * exp(s);
}

// C_n = sqrt(4/pi) Gamma(n+1)/Gamma(n+3/2), the amplitude of the Stieltjes
// expansion; valid for n >= 9 (uses the series at x = n+1 >= 10).
__device__ __forceinline__ double stieltjes_C(double n) {
    return 1.1283791670955126 / gamma_half_ratio_series(n + 1.0);
}

}  // namespace dlt
