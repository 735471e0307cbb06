// Plan construction.  Every parameter is derived from an error bound:
//  * Taylor terms L: smallest even L with (max_k N|dtheta_k|)^L / L! below the
//    truncation budget, max N|dtheta| <= 0.83845 by Lemma 2 (Corollary 2).
//  * Far-field blocks of the Legendre-to-Chebyshev conversion: the remainder
//    of the M-term Stieltjes expansion of P_n(cos theta) is at most
//    2 C_n h_{M,n} / (2 sin theta)^{M+1/2}; a block's first column nlo and its
//    rows are chosen so that this bound stays below the far-field budget at
//    the block's corner (nlo, smallest sin theta), which bounds it everywhere
//    in the block since the bound decreases in n and in sin theta.
//  * Columns n < nd go through the exact dense conversion matrix.
#include "dlt_plan.hpp"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>

#include "dlt_status.h"

namespace dlt {

typedef long double LD;
static const LD PI_L = 3.14159265358979323846264338327950288L;

// Gamma(x+1/2)/Gamma(x), x > 0, in long double: Stirling-type series for
// x >= 20 and the ratio recurrence R(x) = R(x+1) x/(x+1/2) below.
static LD gamma_half_ratio(LD x) {
    static const LD a[] = {-1.0L / 8, 1.0L / 192, -1.0L / 640, 17.0L / 14336, -31.0L / 18432,
                           691.0L / 180224, -5461.0L / 425984, 929569.0L / 15728640};
    LD f = 1.0L;
    while (x < 20) {
        f *= x / (x + 0.5L);
        x += 1;
    }
    LD r = 1.0L / x, r2 = r * r, s = 0, p = r;
    for (int k = 0; k < 8; ++k) {
        s += a[k] * p;
        p *= r2;
    }
    return f * sqrtl(x) * expl(s);
}

// C_n = sqrt(4/pi) Gamma(n+1)/Gamma(n+3/2)
static LD stieltjes_C_host(LD n) { return 2.0L / sqrtl(PI_L) / gamma_half_ratio(n + 1); }

// h_{M,n} = prod_{j=1..M} (j-1/2)^2 / (j (n+j+1/2))
static LD stieltjes_h(int M, LD n) {
    LD h = 1;
    for (int j = 1; j <= M; ++j) h *= (j - 0.5L) * (j - 0.5L) / (j * (n + j + 0.5L));
    return h;
}

// smallest sin(theta) at which the M-term remainder bound at column n is <= eps
static LD far_smin(int M, LD n, LD eps) {
    LD B = 2 * stieltjes_C_host(n) * stieltjes_h(M, n) / eps;
    return 0.5L * powl(B, 1.0L / (M + 0.5L));
}

// first row j (0 <= j < N/2) with sin((j+1/2) pi/N) >= s
static int first_row(int64_t N, LD s) {
    if (s <= 0) return 0;
    if (s >= 1) return (int)(N / 2);
    LD t = asinl(s);
    int64_t j = (int64_t)floorl(t * N / PI_L - 0.5L);
    if (j < 0) j = 0;
    while (j < N / 2 && sinl((j + 0.5L) * PI_L / N) < s) ++j;
    while (j > 0 && sinl((j - 0.5L) * PI_L / N) >= s) --j;
    return (int)j;
}

static int upload(const void* h, size_t bytes, void** d) {
    if (hipMalloc(d, bytes) != hipSuccess) return DLT_ERR_NOMEM;
    if (hipMemcpy(*d, h, bytes, hipMemcpyHostToDevice) != hipSuccess) return DLT_ERR_HIP;
    return 0;
}

static int twiddle_table(int len, LD denom, int mult, cplx** d) {
    std::vector<cplx> t(len > 0 ? len : 1);
    for (int i = 0; i < len; ++i) {
        LD a = 2 * PI_L * (LD)((int64_t)i * mult) / denom;
        t[i].re = (double)cosl(a);
        t[i].im = (double)sinl(a);
    }
    return upload(t.data(), t.size() * sizeof(cplx), (void**)d);
}

// Legendre node parameters: Stieltjes-series Newton for k >= kb, recurrence
// Newton from a Bessel-zero start for k < kb.
static double bessel_j0_zero(int k) {
    // zero k (0-based) of J0: McMahon start, Newton with J0' = -J1
    double b = (k + 0.75) * M_PI;
    double x = b + 1.0 / (8 * b) - 124.0 / (3 * 512 * b * b * b);
    for (int it = 0; it < 8; ++it) x += j0(x) / j1(x);
    return x;
}

// Zeros j_{0,k} of J0 (k = 1..8) and J1 at them.
static const LD BESSEL_J0_ZERO_J1[NODE_CLOSED_KB][2] = {
    {2.404825557695772768622L, 0.5191474972894667881402L},  {5.520078110286310649597L, -0.3402648065583681485649L},
    {8.653727912911012216954L, 0.2714522999283819203881L},  {11.79153443901428161374L, -0.232459831364724778856L},
    {14.93091770848778594776L, 0.2065464330779960268291L},  {18.07106396791092254315L, -0.1877288030404394320809L},
    {21.21163662987925895908L, 0.1732658942292298697358L},  {24.35247153074930273706L, -0.1617015506892500044539L},
};

// Boundary nodes in closed form for N >= NODE_CLOSED_MIN.  u = sqrt(sin t)
// P_N(cos t) solves u'' + (rho^2 + 1/(4 sin^2 t)) u = 0 with rho = N + 1/2,
// and 1/(4 sin^2 t) = 1/(4 t^2) + 1/12 + t^2/60 + ...; dropping the t^2/60
// term leaves Bessel's equation of order 0 in rho' t, rho'^2 = rho^2 + 1/12,
// whose solution regular at 0 with P_N(1) = 1 is sqrt(t) J0(rho' t).  So
// P_N(cos t) = sqrt(t / sin t) J0(rho' t) up to a relative change of order
// t^3 / rho' from the dropped term, below 1e-17 for the first eight nodes
// once N >= 8192: theta_k = j_{0,k+1} / rho' and
// w_k = 2 / (dP_N/dt)^2 = 2 sin(theta_k) / (theta_k rho'^2 J1(j_{0,k+1})^2).
constexpr int64_t NODE_CLOSED_MIN = 8192;
static void closed_boundary_nodes(int64_t N, NodeParams& P) {
    const LD rho2 = ((LD)N + 0.5L) * ((LD)N + 0.5L) + 1.0L / 12;
    const LD rho = sqrtl(rho2);
    for (int k = 0; k < P.kb; ++k) {
        const LD j = BESSEL_J0_ZERO_J1[k][0], J1 = BESSEL_J0_ZERO_J1[k][1];
        const LD t = j / rho;
        P.bd[k] = (double)(t - ((LD)k + 0.5L) * PI_L / (LD)N);
        P.bw[k] = (double)(2 * sinl(t) / (t * rho2 * J1 * J1));
    }
}

void rnode_build(int64_t N, RNode& r) {
    memset(&r, 0, sizeof(r));
    NodeParams& ndp = r.P;
    ndp.N = (int)N;
    ndp.Ms = MAX_NODE_M;
    int nh = (int)((N + 1) / 2);
    ndp.kb = (int)std::min<int64_t>(nh, 6);
    if (N < 128) ndp.kb = nh;
    // the Bessel-zero start is within 2.5 ulp from N = 2048 on (one FP64
    // recurrence Newton step there would add several ulp); below, one step
    ndp.newton_b = (N >= 2048) ? 0 : (N >= 64) ? 1 : 12;
    ndp.C = (double)stieltjes_C_host((LD)N);
    for (int m = 0; m < MAX_NODE_M; ++m) ndp.h[m] = (double)stieltjes_h(m, (LD)N);
    // boundary-node starting offsets from theta^cheb1_k = (k+1/2) pi/N:
    // Bessel-zero form theta ~ psi + (psi cot psi - 1)/(8 psi nu^2),
    // psi = j_{0,k+1}/nu, nu = N+1/2, for N >= 64; else theta^cheb*.
    LD nu = (LD)N + 0.5L;
    for (int k = 0; k < ndp.kb; ++k) {
        LD th;
        if (N >= 64) {
            LD psi = (LD)bessel_j0_zero(k) / nu;
            th = psi + (psi * cosl(psi) / sinl(psi) - 1) / (8 * psi * nu * nu);
        } else {
            th = ((LD)k + 0.75L) * PI_L / nu;
        }
        r.guess[k] = (double)(th - ((LD)k + 0.5L) * PI_L / (LD)N);
    }
    if (N >= NODE_CLOSED_MIN && ndp.kb <= NODE_CLOSED_KB) {
        ndp.closed_b = 1;
        closed_boundary_nodes(N, ndp);
        for (int k = 0; k < ndp.kb; ++k) r.guess[k] = ndp.bd[k];
    }
}

// Geometry and twiddle tables of the length-N DFT (N a power of two)
static int geo_build(int64_t N, Geo& g, cplx** twN1, cplx** twN2, cplx** twHi, cplx** twLo) {
    int lg = 0;
    while ((int64_t(1) << lg) < N) ++lg;
    int l2 = lg / 2, l1 = lg - l2;  // N1 = 2^l1 >= N2 = 2^l2
    int N1 = 1 << l1, N2 = 1 << l2;
    g.N = (int)N;
    g.N1 = N1;
    g.N2 = N2;
    g.colsA = std::min(N1, FFT_CAP / N2);
    g.rowsB = std::min(N2, FFT_CAP / N1);
    g.lrB = 0;
    while ((1 << g.lrB) < g.rowsB) ++g.lrB;
    g.sh = (lg + 1) / 2;
    int rc;
    if ((rc = twiddle_table(N1, N1, 1, twN1))) return rc;
    if ((rc = twiddle_table(N2, N2, 1, twN2))) return rc;
    if ((rc = twiddle_table((int)(N >> g.sh) + 1, (LD)N, 1 << g.sh, twHi))) return rc;
    if ((rc = twiddle_table(1 << g.sh, (LD)N, 1, twLo))) return rc;
    g.twN1 = *twN1;
    g.twN2 = *twN2;
    g.twHi = *twHi;
    g.twLo = *twLo;
    for (int k = 0; k < 4; ++k) {
        const LD a = PI_L * (LD)k / (2 * (LD)N);
        g.qs[k].re = (double)cosl(a);
        g.qs[k].im = (double)sinl(a);
    }
    return 0;
}

int plan_build(int64_t N, int prec, Plan& p, double tol) {
    memset(&p.geo, 0, sizeof(p.geo));
    p.N = N;
    p.prec = prec;
    if (tol > 0 && prec != PREC_FP64) return DLT_ERR_INVALID_ARG;
    p.tol = tol;
    const bool bulk = (prec != PREC_FP64);  // parameters for the 5e-6 budget
    const bool f32 = (prec == PREC_FP32_BULK);
    // ---- FFT geometry
    int rc;
    if ((rc = geo_build(N, p.geo, &p.d_twN1, &p.d_twN2, &p.d_twHi, &p.d_twLo))) return rc;

    // ---- Taylor truncation (Corollary 2 with max N|dtheta| <= 0.83845)
    {
        // 10% of the budget: 5e-14 (FP64), 5e-6 (FP32-bulk, relaxed FP64) or
        // the working tolerance
        const double tolT = (tol > 0) ? tol / 10 : bulk ? 5e-7 : 5e-15;
        int L = 1;
        double f = 0.83845;
        while (f > tolT) {
            ++L;
            f *= 0.83845 / L;
        }
        p.L = (L + 1) & ~1;
    }

    // ---- low-degree block: dense matrix up to DENSE_MAX columns; for large N
    // the block n < N/8 (N/16 at RECURSE_FROM, where that is the dense limit)
    // is itself converted by this algorithm (sub-plan).  Measured at
    // N = 2^20: N/8 is fastest (N/16 +2.5%, N/4 +14%, N/32 +11%: a larger
    // block costs sub-plan work, a smaller one near-field rows and far terms)
    p.nd = (N >= 2 * RECURSE_FROM) ? (int)(N / 8)
           : (N >= RECURSE_FROM)   ? (int)(N / 16)
                                   : (int)std::min<int64_t>(N, DENSE_MAX);
    p.dense_chunk = 512;  // equals DENSE_CH of the dense kernels
    p.dense_nchunk = (p.nd + p.dense_chunk - 1) / p.dense_chunk;
    if (p.nd > DENSE_MAX) {
        p.sub = new Plan();
        if ((rc = plan_build(p.nd, prec, *p.sub, tol))) return rc;
        p.dense_nchunk = 0;
    } else {
        std::vector<double> lam(p.nd);
        for (int z = 0; z < p.nd; ++z) lam[z] = (double)(1.0L / gamma_half_ratio(z + 0.5L));
        if ((rc = upload(lam.data(), lam.size() * sizeof(double), (void**)&p.d_lam))) return rc;
    }

    // ---- far field and near field (only when N > nd)
    FarParams& F = p.far;
    NearParams& Nr = p.near;
    memset(&F, 0, sizeof(F));
    memset(&Nr, 0, sizeof(Nr));
    F.nd = p.nd;
    Nr.nd = p.nd;
    if (N > p.nd) {
        // truncation of the asymptotic series per row, relative to ||c||_1
        // (a working tolerance: 1/50 of it below 1e-11, where rounding takes
        // a share of the budget as in the FP64 mode, else 1/10 as in the
        // 5e-6 modes)
        const LD eps = (tol > 0) ? (LD)tol / (tol < 1e-11 ? 50 : 10) : bulk ? 5e-7L : 1e-15L;
        // cost model (forward + inverse, calibrated on MI355X at N = 2^20):
        // one far term (both passes) ~ 24 us per 2^20 points in FP64, 3/4 of
        // that with FP32 storage; the near field runs 64 rows per wave, so it
        // costs by groups of 64 rows, ~0.8 ps per row-degree in all
        const double far_term_s = (f32 ? 18e-6 : 24e-6) * (double)N / (double)(1 << 20);
        const double near_step_s = 0.8e-12;
        auto near_cost = [&](int rows, int64_t degrees) {
            return (double)(((rows + 63) / 64) * 64) * (double)degrees * near_step_s;
        };
        // terms of the central block: fewest total cost, rows near the ends
        // go to the recurrence
        int M1 = 12;
        {
            double best = 1e300;
            const int mlo = (tol > 0) ? 2 : bulk ? 3 : 8, mhi = (tol > 0) ? 16 : bulk ? 12 : 16;
            for (int m = mlo; m <= mhi; ++m) {
                int j = first_row(N, far_smin(m, p.nd, eps));
                double cost = m * far_term_s + near_cost(j, N - p.nd);
                if (cost < best) {
                    best = cost;
                    M1 = m;
                }
            }
        }
        const int M = M1;
        const double beta = 8.0;
        int half = (int)(N / 2);
        // block 0: central rows, columns n >= nd
        int j0 = first_row(N, far_smin(M1, p.nd, eps));
        F.blk[0] = {j0, half, p.nd, M1};
        F.nblk = 1;
        int jprev = j0;
        // further blocks only where their M full-length transforms cost less
        // than the near-field recurrence they replace
        while (jprev > 0 && F.nblk < MAX_BLOCKS) {
            int jl = (int)floor(jprev / beta);
            LD s = sinl((jl + 0.5L) * PI_L / N);
            // smallest column where M terms are within eps at sin = s
            LD lo = p.nd, hi = (LD)N;
            if (far_smin(M, hi, eps) > s) break;  // no valid column below N
            for (int it = 0; it < 80; ++it) {
                LD mid = 0.5L * (lo + hi);
                if (far_smin(M, mid, eps) <= s) hi = mid; else lo = mid;
            }
            int nlo = (int)ceill(hi);
            if (nlo >= N) break;
            // rows [jl, jprev) keep only degrees [nd, nlo) in the recurrence
            double saved = (double)(jprev - jl) * (double)(N - nlo) * near_step_s;
            if (saved < M * far_term_s) break;
            F.blk[F.nblk++] = {jl, jprev, nlo, M};
            jprev = jl;
        }
        F.Mmax = 0;
        F.nterm = 0;
        for (int b = 0; b < F.nblk; ++b) F.Mmax = std::max(F.Mmax, F.blk[b].M);
        {
            LD hk = 1;
            for (int j = 1; j < F.Mmax; ++j) hk *= (j - 0.5L) * (j - 0.5L) / j;
            F.hK = (double)hk;
        }
        for (int m = 0; m < F.Mmax; ++m)
            for (int b = 0; b < F.nblk; ++b)
                if (m < F.blk[b].M) {
                    if (F.nterm >= MAX_TERMS) return DLT_ERR_UNSUPPORTED;
                    F.term_blk[F.nterm] = b;
                    F.term_m[F.nterm] = m;
                    ++F.nterm;
                }
        // near-field segments: blocks b >= 1 need columns [nd, nlo); rows
        // below the last block need [nd, N)
        Nr.jnear = jprev;  // rows j < jnear: endpoint rows
        int items = 0;
        auto add_seg = [&](int jlo, int jhi, int nend) {
            if (jhi <= jlo || nend <= p.nd) return;
            Seg s;
            s.jlo = jlo;
            s.jhi = jhi;
            s.nend = nend;
            s.nchunk = (nend + NEAR_CHUNK - 1) / NEAR_CHUNK;
            s.item_off = items;
            items += (jhi - jlo) * s.nchunk;
            Nr.seg[Nr.nseg++] = s;
        };
        add_seg(0, jprev, (int)N);
        for (int b = 1; b < F.nblk; ++b) add_seg(F.blk[b].jlo, F.blk[b].jhi, F.blk[b].nlo);
        Nr.nitems = items;
        // work-group tables of the transposed near field (256 rows x one chunk)
        {
            std::vector<int> wgseg, segoff(2 * MAX_SEGS, 0), rgnend;
            int wg = 0, rg = 0;
            for (int s = 0; s < Nr.nseg; ++s) {
                const Seg& S = Nr.seg[s];
                int ng = (S.jhi - S.jlo + 63) / 64;
                segoff[2 * s] = wg;
                segoff[2 * s + 1] = rg;
                for (int i = 0; i < S.nchunk * ng; ++i) wgseg.push_back(s);
                for (int i = 0; i < ng; ++i) rgnend.push_back(S.nend);
                wg += S.nchunk * ng;
                rg += ng;
            }
            p.tn_wg = wg;
            p.tn_nrg = rg;
            if (wg > 0) {
                if ((rc = upload(wgseg.data(), wgseg.size() * sizeof(int), (void**)&p.d_tn_wgseg))) return rc;
                if ((rc = upload(rgnend.data(), rgnend.size() * sizeof(int), (void**)&p.d_tn_rgnend))) return rc;
            }
            if ((rc = upload(segoff.data(), segoff.size() * sizeof(int), (void**)&p.d_tn_segoff))) return rc;
        }
        Nr.jnear = (F.nblk > 1) ? F.blk[1].jhi : jprev;  // rows j < jnear may carry near terms
        if (Nr.nseg == 0) Nr.jnear = 0;
        // 1/(n+1), the recurrence coefficient of the near field
        std::vector<double> R(N);
        for (int64_t n = 0; n < N; ++n) R[n] = (double)(1.0L / (LD)(n + 1));
        if ((rc = upload(R.data(), N * sizeof(double), (void**)&p.d_rcp))) return rc;
    }

    // ---- nodes
    {
        RNode rn;
        rnode_build(N, rn);
        p.nodes = rn.P;
        if ((rc = upload(rn.guess, (size_t)std::max(rn.P.kb, 1) * sizeof(double), (void**)&p.d_guess))) return rc;
    }

    // ---- workspace per instance
    // Taylor pairs: the plan's, or up to RAGGED_Q_MAX for grids shared by
    // smaller sizes (nodes up to half a grid step from their rows)
    const int qmax = bulk ? RAGGED_Q_MAX_BULK : RAGGED_Q_MAX;
    int nX = std::max({F.nterm, p.L / 2, qmax, 1});
    {
        // about 512 (tile, term group) blocks per pass, one round of two per
        // CU: every term group repeats its tiles' per-block set-up (twiddle
        // staging, amplitude or row-factor reads, the first tile), so more
        // groups than needed to fill the GPU cost time (measured at N = 2^20:
        // one group per pass is fastest)
        const Geo& g = p.geo;
        int tilesA = g.N1 / g.colsA, tilesB = g.N2 / g.rowsB;
        int nt = std::max(F.nterm, 1);
        p.tgA = std::min({nt, 16, std::max(1, (512 + tilesA - 1) / tilesA)});
        p.tgB = std::min({nt, 4, std::max(1, (512 + tilesB - 1) / tilesB)});
    }
    p.ws_X = (size_t)nX * N * sizeof(cplx);
    if (f32)  // FP32 far terms; or the FP64 Taylor pair 0 + FP32 pairs 1..Q-1
        p.ws_X = std::max((size_t)std::max(F.nterm, 1) * N * sizeof(cplxf),
                          (size_t)N * sizeof(cplx) + (size_t)(qmax - 1) * N * sizeof(cplxf));
    // the low-degree sub-run has its own region: it runs beside the far field
    p.ws_sub = p.sub ? p.sub->ws_per_inst : 0;
    p.ws_v = (size_t)p.tgB * N * sizeof(double);
    p.ws_items = (size_t)Nr.nitems * 2 * sizeof(double);
    p.ws_near = (size_t)2 * std::max(Nr.jnear, 1) * sizeof(double);
    p.ws_dense = (size_t)(p.dense_nchunk + 1) * p.nd * sizeof(double);
    p.ws_chat = (size_t)N * sizeof(double);
    p.ws_vec = (size_t)N * sizeof(double);
    p.ws_part = (size_t)p.tn_nrg * N * sizeof(double);
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    p.ws_per_inst = al(p.ws_X) + al(p.ws_v) + al(p.ws_items) + al(p.ws_near) + al(p.ws_dense) +
                    al(p.ws_chat) + al(p.ws_vec) + al(p.ws_part) + al(p.ws_sub);
    p.ws_shared = 3 * al((size_t)N * sizeof(double));  // theta, w, dtheta
    return 0;
}

// Taylor terms on the theta^cheb* grid: N |theta_k - theta^cheb*_k| <=
// N/(3 pi (2N+1)) < 1/(6 pi) (Lemma 2), so the truncation error is at most
// ||c||_1 / ((6 pi)^L L!) (Corollary 2, second bound); L is the smallest
// with that factor within a tenth of the FP64 budget, 5e-15 (L = 8).
int star_terms(double tolT) {
    int L = 1;
    double f = 1.0 / (6 * M_PI);
    while (f > tolT) {
        ++L;
        f /= 6 * M_PI * L;
    }
    return L;
}

int star_plan_build(int64_t N, StarPlan& s) {
    s = StarPlan();
    s.N = N;
    s.L = star_terms(5e-15);
    int rc;
    if ((rc = geo_build(2 * N, s.geo, &s.d_twN1, &s.d_twN2, &s.d_twHi, &s.d_twLo))) return rc;
    s.ws_per_inst = ((size_t)s.L * 2 * (size_t)N * sizeof(cplx) + 255) & ~size_t(255);
    return 0;
}

void star_plan_free(StarPlan& s) {
    void* ptrs[] = {s.d_twN1, s.d_twN2, s.d_twHi, s.d_twLo, s.d_H};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    s = StarPlan();
}

void plan_free(Plan& p) {
    if (p.sub) {
        plan_free(*p.sub);
        delete p.sub;
        p.sub = nullptr;
    }
    if (p.star) {
        star_plan_free(*p.star);
        delete p.star;
        p.star = nullptr;
    }
    void* ptrs[] = {p.d_twN1,  p.d_twN2,     p.d_twHi,      p.d_twLo,     p.d_lam,
                    p.d_rcp,   p.d_guess,    p.d_tn_wgseg,  p.d_tn_segoff, p.d_tn_rgnend, p.d_near_st,
                    p.d_amp,   p.d_rowf,     p.d_theta,     p.d_w,        p.d_dth};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    p = Plan();
}

}  // namespace dlt
