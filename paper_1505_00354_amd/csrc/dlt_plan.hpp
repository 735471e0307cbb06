// Host-side plan for one transform size N: FFT geometry, the block split of
// the Legendre-to-Chebyshev conversion, the Taylor truncation L, node
// parameters, device tables, and the workspace layout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "dlt_common.hpp"

namespace dlt {

constexpr int MAX_TERMS = 64;   // far-field (block, m) pairs
constexpr int MAX_BLOCKS = 8;
constexpr int MAX_NODE_M = 24;  // terms of the Stieltjes series for nodes
constexpr int MAX_SEGS = 8;     // near-field row segments
constexpr int NEAR_CHUNK = 512;
constexpr int NEAR_SUB = 128;   // near-field states are kept every NEAR_SUB degrees
constexpr int NEAR_NSUB = NEAR_CHUNK / NEAR_SUB;
constexpr int64_t MAX_N = int64_t(1) << 20;
constexpr int DENSE_MAX = 8192;         // largest low-degree block done by the dense matrix
constexpr int64_t RECURSE_FROM = 1 << 17;  // from this N on the low block is N/16, recursively
// Taylor pairs a grid may run for sizes padded to it (|d| n/Ng <= pi/2):
// L = 20 for 5e-15, L = 12 for 5e-7
constexpr int RAGGED_Q_MAX = 10;
constexpr int RAGGED_Q_MAX_BULK = 6;

// FFT geometry of the length-N DFT (N power of two): N = N1*N2.  Pass A runs
// length-N2 DFTs over the slow input index for tiles of colsA columns; pass B
// runs length-N1 DFTs over the fast input index for tiles of rowsB rows.
struct Geo {
    int N, N1, N2, colsA, rowsB, sh;
    int lrB;  // log2(rowsB)
    const cplx* twN1;  // e^{2 pi i t/N1}
    const cplx* twN2;  // e^{2 pi i t/N2}
    const cplx* twHi;  // e^{2 pi i (t<<sh)/N}
    const cplx* twLo;  // e^{2 pi i t/N}, t < 2^sh
    cplx qs[4];        // e^{i pi k/(2N)}, k < 4
};

// Far-field block b: rows j in [jlo, jhi) and the mirrored rows
// [N-jhi, N-jlo); columns n >= nlo; M terms of the Stieltjes series.
struct Block {
    int jlo, jhi, nlo, M;
};

// Near-field segment: rows j in [jlo, jhi) (and mirrors), recurrence over
// n in [0, nend), contributions accumulated for n >= nd.
struct Seg {
    int jlo, jhi, nend, nchunk;
    int item_off;  // first item of this segment
};

struct FarParams {
    int nblk, nterm, Mmax, nd;
    double hK;  // prod_{j=1}^{Mmax-1} (j-1/2)^2 / j
    Block blk[MAX_BLOCKS];
    // int (not byte) entries so that kernels read them with scalar loads
    int term_blk[MAX_TERMS], term_m[MAX_TERMS];  // ordered by ascending m
    // row -> block lookup: rows j < blk_edge[b] (and mirrors) are outside
    // blocks 0..b-1; block 0 is the central one.
};

struct NearParams {
    int nseg, nitems, jnear, nd;
    Seg seg[MAX_SEGS];
};

constexpr int NODE_CLOSED_KB = 8;  // boundary nodes the closed form may cover
struct NodeParams {
    int N, kb, Ms, newton_b;   // boundary nodes k < kb use the recurrence
    int closed_b;              // 1: boundary nodes k < kb from the closed form (bd, bw)
    double C;                  // C_N of the Stieltjes series
    double h[MAX_NODE_M];      // h_{m,N}
    double bd[NODE_CLOSED_KB]; // closed form: theta_k - (k+1/2) pi/N
    double bw[NODE_CLOSED_KB]; // closed form: w_k
};

// Node parameters of one instance of a ragged batch: its NodeParams and the
// starting offsets of its boundary nodes (kb <= RNODE_GUESS).
constexpr int RNODE_GUESS = 64;
struct RNode {
    NodeParams P;
    double guess[RNODE_GUESS];
};
// Fills `r` for size N (any N >= 1); host only.
void rnode_build(int64_t N, RNode& r);

// Per-instance tables of a ragged batch on the power-of-two grid of size Ng
// (instance b at b*Ng): the node paired with grid row j (or -1), Ng times its
// offset from that row's angle, its weight; and each instance's offset in the
// caller's arrays.  gk == nullptr: the plain layout (node k on row k).
struct RaggedRows {
    const int* gk;
    const double* dg;
    const double* wg;
    const int64_t* offs;
};

// Arithmetic of a plan: FP64 throughout (5e-14 budget); FP32-bulk (the
// far-field terms and Taylor pairs q >= 1 stored and transformed in FP32,
// parameters for a 5e-6 budget; nodes, amplitudes, near field, pair 0,
// Horner and the DCT-II/III stay FP64); or FP64 with the 5e-6 parameters
// (the equal-accuracy FP64 reference for FP32-bulk).
constexpr int PREC_FP64 = 0;
constexpr int PREC_FP32_BULK = 1;
constexpr int PREC_FP64_RELAXED = 2;

// Evaluation on the grid theta^cheb*_k = (k+3/4) pi/(N+1/2) (Sec. 2.2): at
// these points the sums of Sec. 2.3 are odd outputs of length-(2N+1)
// transforms.  Each Taylor term runs as a chirp-z transform: with
// alpha = 2 pi/(2N+1), sum_{n<N} x_n e^{i n (k+3/4) alpha} equals
// e^{i alpha k^2/2} sum_n [x_n e^{i alpha (n^2/2 + 3n/4)}] e^{-i alpha (k-n)^2/2},
// a cyclic convolution of power-of-two length M = 2N (inputs n < N, outputs
// k < N, lags |k - n| < N), done with length-M DFTs.
struct StarPlan {
    int64_t N = 0;
    int L = 8;               // Taylor terms: smallest L with 1/((6 pi)^L L!) <= 5e-15
    Geo geo{};               // the length-M DFT (M = 2N)
    cplx *d_twN1 = nullptr, *d_twN2 = nullptr, *d_twHi = nullptr, *d_twLo = nullptr;
    cplx* d_H = nullptr;     // (1/M) DFT of the cyclic chirp, in the blocked layout
    size_t ws_per_inst = 0;  // L slabs of M complex values
};

struct Plan {
    int64_t N = 0;
    int prec = PREC_FP64;
    // working tolerance of a tolerance plan (FP64 arithmetic, parameters for
    // ||error|| <= tol ||c||_1); 0 for the fixed budgets of the precision modes
    double tol = 0;
    int L = 16;        // Taylor terms (even)
    int nd = 0;        // columns n < nd handled by the dense block
    int dense_chunk = 1024, dense_nchunk = 0;
    Geo geo{};
    FarParams far{};
    NearParams near{};
    NodeParams nodes{};
    // device tables
    cplx *d_twN1 = nullptr, *d_twN2 = nullptr, *d_twHi = nullptr, *d_twLo = nullptr;
    double* d_lam = nullptr;     // Lambda(z), z < nd
    double* d_rcp = nullptr;     // 1/(n+1), n < N (near field)
    double* d_guess = nullptr;   // boundary-node initial offsets from theta^cheb1
    // transposed near field: work-group -> segment table, per-segment
    // (first work-group, first row group), and nend of every row group
    int* d_tn_wgseg = nullptr;
    int* d_tn_segoff = nullptr;
    int* d_tn_rgnend = nullptr;
    int tn_wg = 0, tn_nrg = 0;
    // near-field recurrence state (P_n, D_n) at the start of every (row,
    // chunk) item and every NEAR_SUB degrees inside it: it does not depend on
    // the input, so it is formed once per plan (2 * NEAR_NSUB doubles per item)
    double* d_near_st = nullptr;
    // far-field tables, input-independent, formed once per plan on the
    // device: amp[n] = C_n h_{Mmax-1,n} e^{i pi n/(2N)} (zero for n < nd) and
    // rowf[m] = e^{i(theta_j-pi/2)/2} (2 sin theta_j)^{-1/2} on the Chebyshev
    // grid, for the row j = j(m) of DFT output m (its square is the factor
    // e^{i(theta_j-pi/2)} / (2 sin theta_j) between consecutive terms m)
    cplx* d_amp = nullptr;
    cplx* d_rowf = nullptr;
    // workspace sizes per transform instance (bytes)
    size_t ws_X = 0, ws_v = 0, ws_items = 0, ws_near = 0, ws_dense = 0, ws_chat = 0, ws_vec = 0;
    size_t ws_part = 0, ws_sub = 0;
    size_t ws_per_inst = 0, ws_shared = 0;
    int tgA = 1;       // far-field pass-A term groups (blocks split the terms)
    int tgB = 1;       // far-field pass-B term groups (partial outputs summed later)
    // low-degree block n < nd when nd exceeds the dense limit: the same
    // transform at size nd (owned)
    Plan* sub = nullptr;
    // theta^cheb* evaluation of this size (FP64 plans; built on first use, owned)
    StarPlan* star = nullptr;
    // the Legendre nodes theta_k, weights w_k and offsets theta_k - (k+1/2) pi/N
    // (input-independent: formed on the device once, when a plan that
    // evaluates at the nodes is built; null in sub-plans)
    double *d_theta = nullptr, *d_w = nullptr, *d_dth = nullptr;
};

// Builds the plan for size N (power of two, 1 <= N <= MAX_N) and precision
// `prec`; returns 0 or a DLT status code.  Allocates the device tables.
// With tol > 0 (PREC_FP64 only) the Taylor and far-field truncations are
// set for the working tolerance tol instead of the mode's fixed budget.
int plan_build(int64_t N, int prec, Plan& p, double tol = 0);
void plan_free(Plan& p);
// Host part of the theta^cheb* plan of size N (power of two): geometry,
// twiddle tables, term count and workspace; d_H is formed on the device
// (star_prepare).  Returns 0 or a DLT status code.
int star_plan_build(int64_t N, StarPlan& s);
// Taylor terms about theta^cheb* for a truncation budget tolT (times ||c||_1)
int star_terms(double tolT);
void star_plan_free(StarPlan& s);

}  // namespace dlt
