// Device-side building blocks shared by the DLT kernels: complex arithmetic,
// twiddle access, the LDS-resident FFT, and the Gamma-ratio series used by
// the asymptotic (Stieltjes) expansion of P_n(cos theta).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace dlt {

// Complex value in precision R (double, or float for the FP32-bulk passes).
template <class R>
struct cplxT {
    R re, im;
};
using cplx = cplxT<double>;
using cplxf = cplxT<float>;

template <class R>
__device__ __forceinline__ cplxT<R> cmul(cplxT<R> a, cplxT<R> b) {
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
template <class R>
__device__ __forceinline__ cplxT<R> cadd(cplxT<R> a, cplxT<R> b) {
    return {a.re + b.re, a.im + b.im};
}
template <class R>
__device__ __forceinline__ cplxT<R> csub(cplxT<R> a, cplxT<R> b) {
    return {a.re - b.re, a.im - b.im};
}
template <class R>
__device__ __forceinline__ cplxT<R> cscale(cplxT<R> a, R s) {
    return {a.re * s, a.im * s};
}
template <class R>
__device__ __forceinline__ cplxT<R> cconj(cplxT<R> a) {
    return {a.re, -a.im};
}
// multiply by +i
template <class R>
__device__ __forceinline__ cplxT<R> cmuli(cplxT<R> a) {
    return {-a.im, a.re};
}
// precision changes (round to nearest)
template <class R>
__device__ __forceinline__ cplxT<R> cto(cplx a) {
    return {(R)a.re, (R)a.im};
}
template <class R>
__device__ __forceinline__ cplx cwide(cplxT<R> a) {
    return {(double)a.re, (double)a.im};
}

// Threads per block of every FFT-carrying kernel, and the number of complex
// values in one block's tile (32 KiB).
constexpr int FFT_THREADS = 256;
constexpr int FFT_CAP = 2048;
constexpr int FFT_VPT = FFT_CAP / FFT_THREADS;  // tile elements per thread
// LDS slots of a run-time-length tile: one pad slot per 8 values plus a
// per-sequence skew.  A compile-time length swizzles its slots instead and
// needs exactly FFT_CAP of them.
constexpr int FFT_LDS = FFT_CAP + FFT_CAP / 8 + 32;
#define TILE_LDS(L) ((L) > 0 ? FFT_CAP : FFT_LDS)
__device__ __forceinline__ int lp(int x) { return x + (x >> 3); }

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
// then writes, so one buffer suffices.  Used for lengths below 64 only.
template <class R>
__device__ inline void lds_fft(cplxT<R>* buf, int len, int cols, const cplxT<R>* __restrict__ tw) {
    const int tid = threadIdx.x;
    for (int p = 1; p < len;) {
        const int r = ((len / p) & 3) == 0 ? 4 : 2;
        const int nb = len / r;
        const int total = nb * cols;
        const int tstride = len / (p * r);
        cplxT<R> v[FFT_VPT];
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
                    cplxT<R> x0 = buf[lp(cb0 + i)], x1 = buf[lp(cb0 + i + nb)], x2 = buf[lp(cb0 + i + 2 * nb)],
                         x3 = buf[lp(cb0 + i + 3 * nb)];
                    if (p > 1) {
                        cplxT<R> w1 = tw[k * tstride];
                        cplxT<R> w2 = cmul(w1, w1);
                        cplxT<R> w3 = cmul(w2, w1);
                        x1 = cmul(x1, w1);
                        x2 = cmul(x2, w2);
                        x3 = cmul(x3, w3);
                    }
                    cplxT<R> s02 = cadd(x0, x2), d02 = csub(x0, x2);
                    cplxT<R> s13 = cadd(x1, x3), d13 = cmuli(csub(x1, x3));
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
                    cplxT<R> x0 = buf[lp(cb0 + i)], x1 = buf[lp(cb0 + i + nb)];
                    if (p > 1) x1 = cmul(x1, tw[k * tstride]);
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

// In-place length-8 DFT with the + sign, a_q <- sum_j a_j e^{2 pi i j q/8}:
// one radix-2 split (a_j +- a_{j+4}, the difference turned by e^{2 pi i j/8})
// followed by two length-4 DFTs giving the even and the odd outputs.
template <class R>
__device__ __forceinline__ void dft8(cplxT<R>* a) {
    const R h = (R)0.70710678118654752440;  // 1/sqrt(2)
    cplxT<R> b0 = cadd(a[0], a[4]), b1 = cadd(a[1], a[5]), b2 = cadd(a[2], a[6]), b3 = cadd(a[3], a[7]);
    cplxT<R> c0 = csub(a[0], a[4]), c1 = csub(a[1], a[5]), c2 = csub(a[2], a[6]), c3 = csub(a[3], a[7]);
    c1 = {(c1.re - c1.im) * h, (c1.re + c1.im) * h};     // * e^{i pi/4}
    c2 = cmuli(c2);                                       // * e^{i pi/2}
    c3 = {-(c3.re + c3.im) * h, (c3.re - c3.im) * h};    // * e^{3 i pi/4}
    cplxT<R> s02 = cadd(b0, b2), d02 = csub(b0, b2), s13 = cadd(b1, b3), d13 = cmuli(csub(b1, b3));
    cplxT<R> t02 = cadd(c0, c2), e02 = csub(c0, c2), t13 = cadd(c1, c3), e13 = cmuli(csub(c1, c3));
    a[0] = cadd(s02, s13);
    a[2] = cadd(d02, d13);
    a[4] = csub(s02, s13);
    a[6] = csub(d02, d13);
    a[1] = cadd(t02, t13);
    a[3] = cadd(e02, e13);
    a[5] = csub(t02, t13);
    a[7] = csub(e02, e13);
}

// Ownership of the elements of an FFT tile (FFT_CAP values: `cols` sequences
// of length `len`, cols*len = FFT_CAP) among the FFT_THREADS threads.
// Compile-time length L >= 64: thread t owns sequence col = t % cols and the
// 8 indices i0 + s*L/8 (i0 = t / cols), which are exactly the inputs of one
// radix-8 butterfly of the first Stockham stage and the outputs of one
// butterfly of the last, so both stages run in registers.  L == 0 (lengths
// below 64, tiles smaller than FFT_CAP): element e = t + s*FFT_THREADS is
// (e % cols, e / cols) and may lie beyond the tile (live() false).
// Slot swizzle of a compile-time tile of length 2^LOG (6 <= LOG <= 11): for
// every term (i, j), j > i, bit i of the slot is flipped by bit j of the
// element index col*L + i.  Flips of low bits by higher ones make a bijection
// of [0, FFT_CAP), so no padding is needed.  The terms put the lane bits that
// vary within each access of tile_fft on distinct banks, given how gfx950
// serves 16-byte (and 8-byte) LDS accesses, measured with a probe: reads 32
// and 64 lanes at a time, writes 8 and 16 lanes at a time (16-byte slots of
// 64 four-byte banks, a slot's bank group being its index modulo the group
// size).  Every access of tile_fft is then free of bank conflicts.
constexpr int TILE_SWZ_MAX = 7;
constexpr signed char TILE_SWZ[6][TILE_SWZ_MAX][2] = {
    {{0, 8}, {1, 6}, {2, 7}, {3, 9}, {4, 10}, {5, 8}, {-1, -1}},         // L = 64
    {{0, 7}, {1, 9}, {2, 8}, {3, 10}, {4, 7}, {5, 9}, {-1, -1}},         // L = 128
    {{0, 8}, {1, 10}, {2, 9}, {3, 8}, {4, 10}, {5, 9}, {-1, -1}},        // L = 256
    {{0, 3}, {1, 4}, {1, 10}, {2, 9}, {3, 10}, {4, 9}, {5, 10}},         // L = 512
    {{0, 4}, {1, 3}, {2, 5}, {2, 10}, {3, 10}, {4, 10}, {5, 10}},        // L = 1024
    {{0, 5}, {1, 3}, {2, 4}, {3, 6}, {-1, -1}, {-1, -1}, {-1, -1}},      // L = 2048
};
__host__ __device__ constexpr int tile_swizzle(int log_len, int x) {
    int y = x;
    for (int t = 0; t < TILE_SWZ_MAX; ++t) {
        const int i = TILE_SWZ[log_len - 6][t][0], j = TILE_SWZ[log_len - 6][t][1];
        if (i >= 0) y ^= (x >> (j - i)) & (1 << i);
    }
    return y;
}

template <int L>
struct Tile {
    static constexpr int LOG = __builtin_ctz(L);
    static_assert(LOG >= 6 && LOG <= 11, "compile-time tile lengths are 64..2048");
    static constexpr int COLS = FFT_CAP / L;
    static constexpr int STRIDE = L / 8;
    // Stockham stages: radix 8 in registers, NMID radix-8 stages through
    // LDS (p = 8, 64, ...), a last radix-2^RL stage in registers
    static constexpr int RL = ((LOG - 3) % 3) ? (LOG - 3) % 3 : 3;
    static constexpr int NMID = (LOG - 3 - RL) / 3;
    int col_, i0_, rb_;
    __device__ __forceinline__ Tile(int /*cols*/, int /*len*/)
        : col_((int)threadIdx.x % COLS), i0_((int)threadIdx.x / COLS), rb_(sw(col_ * L + i0_)) {}
    __device__ __forceinline__ int col(int) const { return col_; }
    __device__ __forceinline__ int idx(int s) const { return i0_ + s * STRIDE; }
    __device__ __forceinline__ bool live(int) const { return true; }
    __device__ __forceinline__ int cols() const { return COLS; }
    __device__ __forceinline__ int len() const { return L; }
    // LDS slot of element index x (= col*L + i)
    __host__ __device__ static constexpr int sw(int x) { return tile_swizzle(LOG, x); }
    // slot of (col_, idx(s)): the base bits (below STRIDE, and the column)
    // and s*STRIDE are disjoint, so the swizzle splits into two XORed parts,
    // the second a compile-time constant once s is
    __device__ __forceinline__ int slot(int s) const { return rb_ ^ sw(s * STRIDE); }
};

template <>
struct Tile<0> {
    int cols_, len_;
    __device__ __forceinline__ Tile(int cols, int len) : cols_(cols), len_(len) {}
    __device__ __forceinline__ int e(int s) const { return (int)threadIdx.x + s * FFT_THREADS; }
    __device__ __forceinline__ int col(int s) const { return e(s) % cols_; }
    __device__ __forceinline__ int idx(int s) const { return e(s) / cols_; }
    __device__ __forceinline__ bool live(int s) const { return e(s) < cols_ * len_; }
    __device__ __forceinline__ int cols() const { return cols_; }
    __device__ __forceinline__ int len() const { return len_; }
    __device__ __forceinline__ static int sw(int x) { return lp(x); }
    __device__ __forceinline__ int slot(int s) const { return lp(col(s) * len_ + idx(s)); }
};

// Twiddles of the LDS stages of a compile-time length L, stored after the
// L/2 entries e^{2 pi i t/L} of the staged table: for the stage with span p,
// p entries [k] = e^{2 pi i k L/(8p) / L}, k < p.  Lanes of a stage read
// consecutive k, free of bank conflicts (the plain table's indices k L/(8p)
// are multiples of a large power of two).  The higher powers are formed by
// products: LDS bandwidth, not arithmetic, bounds the tile transform.
template <int L>
constexpr int tw_mid_size() {
    if constexpr (L < 64) {
        return 0;
    } else {
        int n = 0;
        for (int st = 0, p = 8; st < Tile<L>::NMID; ++st, p *= 8) n += p;
        return n;
    }
}
template <int L>
constexpr int tw_mid_off(int st) {
    int n = 0;
    for (int i = 0, p = 8; i < st; ++i, p *= 8) n += p;
    return n;
}

// Multiplies a[1..7] by w^1..w^7, w = *w1 (w^2 = w w, w^3 = w^2 w,
// w^4 = w^2 w^2, w^{4+j} = w^4 w^j).
template <class R>
__device__ __forceinline__ void twiddle8_tab(cplxT<R>* a, const cplxT<R>* __restrict__ w1p) {
    const cplxT<R> w1 = *w1p;
    const cplxT<R> w2 = cmul(w1, w1), w3 = cmul(w2, w1), w4 = cmul(w2, w2);
    a[1] = cmul(a[1], w1);
    a[2] = cmul(a[2], w2);
    a[3] = cmul(a[3], w3);
    a[4] = cmul(a[4], w4);
    a[5] = cmul(a[5], cmul(w4, w1));
    a[6] = cmul(a[6], cmul(w4, w2));
    a[7] = cmul(a[7], cmul(w4, w3));
}

// Multiplies a[1..7] by w^1..w^7, w = tw[t] (e^{2 pi i t/L}), the powers
// formed from w as in twiddle8_tab.
template <class R>
__device__ __forceinline__ void twiddle8(cplxT<R>* a, const cplxT<R>* __restrict__ tw, int t) {
    twiddle8_tab(a, tw + t);
}

// Last Stockham stage of a compile-time length L (radix 2^RL, p = L /
// 2^RL) in registers: butterfly index k = i < p with i = i0 + s*STRIDE.
template <int L, class R>
__device__ __forceinline__ void tile_last(cplxT<R>* v, const cplxT<R>* __restrict__ tw, int i0) {
    using TT = Tile<L>;
    constexpr int ST = TT::STRIDE;
    constexpr int RL = TT::RL;
    if constexpr (RL == 3) {
        twiddle8(v, tw, i0);
        dft8(v);
    } else if constexpr (RL == 2) {
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            const int i = i0 + sp * ST;
            cplxT<R> w1 = tw[i];
            cplxT<R> w2 = cmul(w1, w1), w3 = cmul(w1, w2);
            cplxT<R> x0 = v[sp], x1 = cmul(v[sp + 2], w1), x2 = cmul(v[sp + 4], w2), x3 = cmul(v[sp + 6], w3);
            cplxT<R> s02 = cadd(x0, x2), d02 = csub(x0, x2);
            cplxT<R> s13 = cadd(x1, x3), d13 = cmuli(csub(x1, x3));
            v[sp] = cadd(s02, s13);
            v[sp + 2] = cadd(d02, d13);
            v[sp + 4] = csub(s02, s13);
            v[sp + 6] = csub(d02, d13);
        }
    } else {
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
            cplxT<R> x1 = cmul(v[sp + 4], tw[i0 + sp * ST]);
            cplxT<R> x0 = v[sp];
            v[sp] = cadd(x0, x1);
            v[sp + 4] = csub(x0, x1);
        }
    }
}

// DFT with the + sign of every sequence of the tile, v[s] holding the element
// (col(s), idx(s)) on entry and the transform at the same position on exit.
// `buf` is TILE_LDS(L) slots of LDS, `tw` the table e^{2 pi i t/L}, t < L/2,
// followed (compile-time L) by the stage table of tw_mid_size<L>() entries
// (both as staged by stage_twiddles).
// Stockham stages: radix 8 in registers, radix 8 through LDS, and a last
// radix-8/4/2 stage in registers; all threads of the block must call it.  On
// return `buf` is free for reuse (the last LDS reads are behind a barrier).
// `hook(pt)` runs after the barrier of LDS exchange pt, pt = 0 ..
// tile_hook_points<L>() - 1 (a place to issue other work, such as the stores
// of the previous tile, while the exchanges of this one proceed).
struct NoHook {
    __device__ __forceinline__ void operator()(int) const {}
};
template <int L>
constexpr int tile_hook_points() {
    if constexpr (L == 0) return 1;
    else return Tile<L>::NMID + 1;
}
template <int L, class R, class H = NoHook>
__device__ __forceinline__ void tile_fft(cplxT<R>* v, cplxT<R>* buf, const cplxT<R>* __restrict__ tw, const Tile<L>& T,
                                         const H& hook = H()) {
    if constexpr (L == 0) {
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s)
            if (T.live(s)) buf[T.slot(s)] = v[s];
        __syncthreads();
        hook(0);
        lds_fft(buf, T.len(), T.cols(), tw);
#pragma unroll
        for (int s = 0; s < FFT_VPT; ++s)
            if (T.live(s)) v[s] = buf[T.slot(s)];
        __syncthreads();
    } else {
        using TT = Tile<L>;
        constexpr int ST = TT::STRIDE;
        constexpr int NMID = TT::NMID;
        const int cb = T.col_ * L;
        const int i0 = T.i0_;
        // Every slot below is sw(base) ^ sw(offset): the offset's bits lie
        // above the base's within the sequence (8 i0 + q, q < 8; i0 < ST;
        // d's low bits below p, q p from p up to 8 p).
        // first stage (p = 1): no twiddles, outputs to 8 i0 + q
        dft8(v);
        const int wb = TT::sw(cb + 8 * i0);
#pragma unroll
        for (int q = 0; q < 8; ++q) buf[wb ^ TT::sw(q)] = v[q];
        __syncthreads();
        hook(0);
#pragma unroll
        for (int st = 0; st < NMID; ++st) {
            const int p = 8 << (3 * st);
            const int k = i0 & (p - 1);
            cplxT<R> a[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = buf[T.rb_ ^ TT::sw(j * ST)];
            twiddle8_tab(a, tw + L / 2 + tw_mid_off<L>(st) + k);
            dft8(a);
            __syncthreads();
            const int db = TT::sw(cb + (i0 - k) * 8 + k);
#pragma unroll
            for (int q = 0; q < 8; ++q) buf[db ^ TT::sw(q * p)] = a[q];
            __syncthreads();
            hook(st + 1);
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = buf[T.rb_ ^ TT::sw(s * ST)];
        __syncthreads();
        tile_last<L>(v, tw, i0);
    }
}

// tile_fft for a compile-time length that also returns, in vp, the outputs
// of another thread's position (column colp, first index i0p: vp[s] is the
// output at i0p + s L/8 of that column), by reading that thread's inputs to
// the last stage as well and repeating its last stage in registers.
template <int L, class R>
__device__ __forceinline__ void tile_fft_with(cplxT<R>* v, cplxT<R>* vp, cplxT<R>* buf,
                                              const cplxT<R>* __restrict__ tw, const Tile<L>& T, int colp, int i0p) {
    static_assert(L > 0, "compile-time tile lengths only");
    using TT = Tile<L>;
    constexpr int ST = TT::STRIDE;
    constexpr int NMID = TT::NMID;
    const int cb = T.col_ * L;
    const int i0 = T.i0_;
    dft8(v);
    const int wb = TT::sw(cb + 8 * i0);
#pragma unroll
    for (int q = 0; q < 8; ++q) buf[wb ^ TT::sw(q)] = v[q];
    __syncthreads();
#pragma unroll
    for (int st = 0; st < NMID; ++st) {
        const int p = 8 << (3 * st);
        const int k = i0 & (p - 1);
        cplxT<R> a[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = buf[T.rb_ ^ TT::sw(j * ST)];
        twiddle8_tab(a, tw + L / 2 + tw_mid_off<L>(st) + k);
        dft8(a);
        __syncthreads();
        const int db = TT::sw(cb + (i0 - k) * 8 + k);
#pragma unroll
        for (int q = 0; q < 8; ++q) buf[db ^ TT::sw(q * p)] = a[q];
        __syncthreads();
    }
    const int rbp = TT::sw(colp * L + i0p);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        v[s] = buf[T.rb_ ^ TT::sw(s * ST)];
        vp[s] = buf[rbp ^ TT::sw(s * ST)];
    }
    __syncthreads();
    tile_last<L>(v, tw, i0);
    tile_last<L>(vp, tw, i0p);
}

// tile_fft of two independent tiles (v1 in buf1, v2 in buf2, the same
// sequence geometry and table): every stage runs for both before its
// barrier, so a block waits at half the barriers per tile and each wave
// has two independent streams of butterflies and LDS accesses.
template <int L, class R>
__device__ __forceinline__ void tile_fft2(cplxT<R>* v1, cplxT<R>* v2, cplxT<R>* buf1, cplxT<R>* buf2,
                                          const cplxT<R>* __restrict__ tw, const Tile<L>& T) {
    if constexpr (L == 0) {
        tile_fft<L>(v1, buf1, tw, T);
        tile_fft<L>(v2, buf2, tw, T);
    } else {
        using TT = Tile<L>;
        constexpr int ST = TT::STRIDE;
        constexpr int NMID = TT::NMID;
        const int cb = T.col_ * L;
        const int i0 = T.i0_;
        dft8(v1);
        dft8(v2);
        const int wb = TT::sw(cb + 8 * i0);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            buf1[wb ^ TT::sw(q)] = v1[q];
            buf2[wb ^ TT::sw(q)] = v2[q];
        }
        __syncthreads();
#pragma unroll
        for (int st = 0; st < NMID; ++st) {
            const int p = 8 << (3 * st);
            const int k = i0 & (p - 1);
            const cplxT<R>* w1p = tw + L / 2 + tw_mid_off<L>(st) + k;
            cplxT<R> a1[8], a2[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                a1[j] = buf1[T.rb_ ^ TT::sw(j * ST)];
                a2[j] = buf2[T.rb_ ^ TT::sw(j * ST)];
            }
            twiddle8_tab(a1, w1p);
            dft8(a1);
            twiddle8_tab(a2, w1p);
            dft8(a2);
            __syncthreads();
            const int db = TT::sw(cb + (i0 - k) * 8 + k);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                buf1[db ^ TT::sw(q * p)] = a1[q];
                buf2[db ^ TT::sw(q * p)] = a2[q];
            }
            __syncthreads();
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            v1[s] = buf1[T.rb_ ^ TT::sw(s * ST)];
            v2[s] = buf2[T.rb_ ^ TT::sw(s * ST)];
        }
        __syncthreads();
        tile_last<L>(v1, tw, i0);
        tile_last<L>(v2, tw, i0);
    }
}

// Stage twiddles e^{2 pi i t/len}, t < len/2, in the LDS array `stw` of the
// kernel (declared with STAGE_TW) when the length is a compile-time L; the
// FP32 table is the FP64 one rounded.  A run-time length (L == 0) reads the
// global FP64 table directly, or copies len/2 rounded values for FP32.
#define STAGE_TW(name, L, R) \
    __shared__ cplxT<R> name[(L) > 1 ? (L) / 2 + tw_mid_size<L>() : (sizeof(R) == sizeof(double) ? 1 : FFT_CAP / 2)]
template <int L, class R>
__device__ __forceinline__ const cplxT<R>* stage_twiddles(cplxT<R>* stw, const cplx* __restrict__ src, int len) {
    if constexpr (L > 1) {
#pragma unroll
        for (int i = threadIdx.x; i < L / 2; i += FFT_THREADS) stw[i] = cto<R>(src[i]);
        // stage tables: entry (st, k) is e^{2 pi i k (L/(8p))/L}, an index
        // below L/8 of the plain table
        for (int i = threadIdx.x; i < tw_mid_size<L>(); i += FFT_THREADS) {
            int p = 8, k = i;  // stage span p and the index inside its table
            while (k >= p) {
                k -= p;
                p *= 8;
            }
            stw[L / 2 + i] = cto<R>(src[k * (L / (8 * p))]);
        }
        __syncthreads();
        return stw;
    } else if constexpr (sizeof(R) == sizeof(double)) {
        return (const cplxT<R>*)src;
    } else {
        for (int i = threadIdx.x; i < len / 2; i += FFT_THREADS) stw[i] = cto<R>(src[i]);
        __syncthreads();
        return stw;
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
