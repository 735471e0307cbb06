/*
 * dlt.h -- C ABI of the MI355X (gfx950) fast discrete Legendre transform.
 *
 * Implements the transforms of N. Hale and A. Townsend, "A fast FFT-based
 * discrete Legendre transform" (IMA J. Numer. Anal. 36 (2016)):
 *
 *   DLT   (eq. (1))  f_k = sum_{n<N} c_n P_n(x_k),                 0 <= k < N
 *   IDLT  (eq. (2))  c_n = (n+1/2) sum_{k<N} w_k f_k P_n(x_k),     0 <= n < N
 *   NDCT  (eq. (3))  f_k = sum_{n<N} chat_n T_n(x_k)
 *   leg2cheb (Sec. 3, eq. (9))  chat = M c, the Legendre-to-Chebyshev
 *         coefficient map, so that sum c_n P_n = sum chat_n T_n
 *
 * where x_k = cos(theta_k) are the roots of P_N ordered 1 > x_0 > ... >
 * x_{N-1} > -1 (increasing theta_k) and w_k the Gauss-Legendre weights.
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers to double, owned by the caller.
 *     Inputs are never modified.  Outputs must not overlap inputs.
 *   - Batched layout: instance b of a batch occupies elements [b*N, (b+1)*N)
 *     (contiguous, batch-major).
 *   - Calls are asynchronous on `stream` (0 = default stream); the library
 *     does not synchronise.  Errors of kernels already enqueued surface as
 *     DLT_ERR_HIP from a later call or from the caller's own synchronisation.
 *   - batch == 0 is a no-op returning DLT_OK.
 *   - Supported sizes: 1 <= N <= DLT_MAX_N (larger N return
 *     DLT_ERR_UNSUPPORTED).  Powers of two run on the Chebyshev grid of the
 *     same size; other N run on the next power-of-two grid, with the inputs
 *     zero-padded and every Legendre node paired with its nearest grid point
 *     (more Taylor terms, same accuracy).
 *   - The library keeps per-N plans (twiddle and coefficient tables, the
 *     input-independent near-field recurrence states, and the nodes, weights
 *     and offsets theta_k - (k+1/2) pi/N, all formed on the device)
 *     and a per-stream workspace; both are created on first use and live
 *     until dlt_release() or process exit.  The first call for a given N on
 *     a device builds its plan and synchronises the device (so it must not
 *     be made inside stream capture); a call that needs a larger workspace
 *     than its stream holds synchronises that stream before replacing it;
 *     other calls never synchronise.  Calls on different streams use
 *     different workspaces and may run at the same time.
 *   - Repeated calls: when leg2cheb, cheb_eval_leggrid, dlt_forward,
 *     dlt_inverse, cheb2leg (and their _ex and _tol forms), leg2chebvals or
 *     chebvals2leg are called again with the same size
 *     (a power of two), batch, precision, buffers and stream, the second
 *     call captures its work into a HIP graph (on a library-owned stream)
 *     and it and later such calls launch that graph on `stream`: the same
 *     kernels on the buffers' current contents, the same results.  Calls
 *     made while the kernel trace is on, and the first call, run directly;
 *     with DLT_CALL_GRAPHS=0 in the environment (read at the first call)
 *     every call runs directly.  dlt_release() frees the graphs.
 *   - FP64 arithmetic throughout.  Accuracy against the direct O(N^2)
 *     definitions: max_k |f_k - f_k^exact| <= 5e-14 * sum_n |c_n| (DLT, NDCT);
 *     max_n |c_n - c_n^exact| <= 5e-14 * (n+1/2) sum_k w_k |f_k| (IDLT).
 *
 * Status codes (int return value of every call)
 */
#ifndef DLT_H_
#define DLT_H_

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DLT_OK 0
#define DLT_ERR_INVALID_ARG (-1) /* N < 1, batch < 0, NULL pointer, overlapping in/out */
#define DLT_ERR_UNSUPPORTED (-2) /* N > DLT_MAX_N (plan queries: N not a power of two) */
#define DLT_ERR_HIP (-3)         /* a HIP runtime call or kernel launch failed */
#define DLT_ERR_NOMEM (-4)       /* device workspace or plan tables could not be allocated */
#define DLT_ERR_NOT_PREPARED (-5) /* dlt_forward_noalloc: the size's plan has not been built */

#define DLT_MAX_N (1LL << 20)

/* Legendre nodes and weights (Sec. 1; theta form, Sec. 2.1-2.2).
 * theta[k] = arccos(x_k) (increasing), w[k] = w_k, dtheta[k] =
 * theta_k - (k+1/2) pi/N (offset from the Chebyshev points of the first kind,
 * computed directly rather than by subtraction).  Any of the three outputs
 * may be NULL to skip it; `batch` copies of each output are written. */
int leg_nodes_weights(int64_t N, int64_t batch, double* theta, double* w, double* dtheta, hipStream_t stream);

/* Legendre-to-Chebyshev coefficients chat = M c (Sec. 3, eq. (9)), c and chat
 * each of length N per instance. */
int leg2cheb(int64_t N, int64_t batch, const double* c, double* chat, hipStream_t stream);

/* Chebyshev expansion sum_n chat_n T_n evaluated at the N Legendre nodes,
 * eq. (3) (the "NDCT" of Sec. 2). */
int cheb_eval_leggrid(int64_t N, int64_t batch, const double* chat, double* f, hipStream_t stream);

/* Discrete Legendre transform, eq. (1). */
int dlt_forward(int64_t N, int64_t batch, const double* c, double* f, hipStream_t stream);

/* Inverse discrete Legendre transform, eq. (2) (Sec. 4). */
int dlt_inverse(int64_t N, int64_t batch, const double* f, double* c, hipStream_t stream);

/* Chebyshev expansion at near-Chebyshev points (the NDCT of Sec. 2, eq. (3),
 * at theta_k = (k+1/2) pi/N + dtheta_k): f_k = sum_n chat_n cos(n theta_k),
 * by the same Taylor series in the offsets (Sec. 2.1, Cor. 1) as
 * cheb_eval_leggrid, for points such as Gauss-Jacobi nodes (Sec. 1 names the
 * Hankel-transform analogue).  dtheta: N offsets (device, shared by every
 * batch instance), same convention as leg_nodes_weights's dtheta.
 * Precondition: |N dtheta_k| <= pi/2 for every k; the Taylor length (L = 20)
 * is chosen for that bound, so the error is at most 5e-14 ||chat||_1 as for
 * cheb_eval_leggrid.  An output f_k whose offset exceeds the bound
 * (|N dtheta_k| > (pi/2)(1 + 1e-12)) is NaN; the call still returns DLT_OK
 * (the offsets are device data, read only by the kernels).  N must be a
 * power of two (DLT_ERR_UNSUPPORTED otherwise); dtheta must not overlap f.
 * Calls are never captured into a graph. */
int cheb_eval_nodes(int64_t N, int64_t batch, const double* chat, const double* dtheta, double* f,
                    hipStream_t stream);

/* Legendre coefficients <-> values at the Chebyshev points x_j =
 * cos((j+1/2) pi/N), j = 0..N-1 (decreasing x, the order of the Legendre
 * outputs) (Sec. 1, the arcs of Fig. 1 between Legendre coefficients and
 * values on a Chebyshev grid):
 *   leg2chebvals  v_j = sum_n c_n P_n(x_j): leg2cheb, then the Chebyshev
 *                 expansion on the grid (a DCT-III);
 *   chebvals2leg  c = the Legendre coefficients of the polynomial of degree
 *                 < N through the values v_j: the Chebyshev coefficients of
 *                 the interpolant (a DCT-II, chat_n = (eps_n/N) sum_j v_j
 *                 cos(n theta_j)), then cheb2leg; c is used as the
 *                 intermediate for the values at the Legendre nodes.
 * Accuracy: leg2chebvals as dlt_forward, ||v - v^exact||_inf <= 5e-14
 * ||c||_1; chebvals2leg as cheb2leg applied to the exact Chebyshev
 * coefficients chat of the interpolant, max_n |c_n - c_n^exact| /
 * ((n+1/2) ||chat||_1) <= 2e-13.  FP64; N must be a power of two
 * (DLT_ERR_UNSUPPORTED otherwise); other arguments and errors as for
 * leg2cheb. */
int leg2chebvals(int64_t N, int64_t batch, const double* c, double* v, hipStream_t stream);
int chebvals2leg(int64_t N, int64_t batch, const double* v, double* c, hipStream_t stream);

/* Chebyshev-to-Legendre coefficients c = M^{-1} chat (the inverse of
 * leg2cheb, Sec. 3): the Chebyshev expansion is evaluated at the Legendre
 * nodes (as cheb_eval_leggrid) and the inverse transform (as dlt_inverse)
 * is applied to those values, which is exact for degree < N because the
 * Gauss-Legendre rule integrates P_n T_m exactly for n + m <= 2N - 1
 * (Sec. 4, eq. (10)).  c is used as the intermediate for the values.
 * Accuracy: max_n |c_n - c_n^exact| / ((n+1/2) ||chat||_1) <= 2e-13 (the
 * evaluation's and the inverse's errors added).  Arguments, layout, sizes
 * and errors as for leg2cheb. */
int cheb2leg(int64_t N, int64_t batch, const double* chat, double* c, hipStream_t stream);

/* Arithmetic of the _ex entry points (FP64 inputs and outputs in both).
 *   DLT_PREC_FP64       the plain method in FP64 (what the entry points above
 *                       use): accuracy as stated at the top of this file.
 *   DLT_PREC_FP32_BULK  the far-field terms and the Taylor pairs l >= 2 are
 *                       stored and transformed in FP32 (half the bytes of
 *                       those intermediates), with the method's parameters
 *                       chosen for a 5e-6 budget (fewer far-field terms,
 *                       L = 10 Taylor terms); nodes, dtheta, the asymptotic
 *                       amplitudes, the near field, the low-degree block, the
 *                       l = 0, 1 Taylor pair, the Horner sums and the
 *                       DCT-II/III stay FP64.  Accuracy: the norms above
 *                       within 5e-6 instead of 5e-14.
 *   DLT_PREC_FP64_RELAXED  FP64 arithmetic with the FP32-bulk parameters
 *                       (same 5e-6 budget): the plain method at equal stated
 *                       accuracy, for comparisons with DLT_PREC_FP32_BULK.
 * Any other value returns DLT_ERR_INVALID_ARG. */
#define DLT_PREC_FP64 0
#define DLT_PREC_FP32_BULK 1
#define DLT_PREC_FP64_RELAXED 2

/* leg2cheb, cheb_eval_leggrid, dlt_forward, dlt_inverse and cheb2leg with a
 * precision mode (DLT_PREC_*); same arguments and behaviour otherwise. */
int leg2cheb_ex(int64_t N, int64_t batch, const double* c, double* chat, int prec, hipStream_t stream);
int cheb_eval_leggrid_ex(int64_t N, int64_t batch, const double* chat, double* f, int prec, hipStream_t stream);
int dlt_forward_ex(int64_t N, int64_t batch, const double* c, double* f, int prec, hipStream_t stream);
int dlt_inverse_ex(int64_t N, int64_t batch, const double* f, double* c, int prec, hipStream_t stream);
int cheb2leg_ex(int64_t N, int64_t batch, const double* chat, double* c, int prec, hipStream_t stream);

/* The same five operations for a working tolerance eps (Sec. 3: every
 * parameter of the method follows from the accuracy goal; Sec. 2, Cor. 1 and
 * Table 1 for the Taylor terms).  FP64 arithmetic; the Taylor length and the
 * far-field terms, blocks and rows (hence the near field) are chosen for eps
 * instead of the fixed 5e-14 / 5e-6 budgets of the precision modes, so the
 * accuracy statements at the top of this file hold with eps in place of
 * 5e-14.  eps is rounded down to the steps 1, 2, 5 x 10^e from 5e-14 to 1e-1
 * (one cached plan per step and N).  N must be a power of two
 * (DLT_ERR_UNSUPPORTED otherwise); eps outside [5e-14, 1e-1] or NaN gives
 * DLT_ERR_INVALID_ARG; arguments, layout, ownership and the other errors as
 * for the plain entry points. */
int leg2cheb_tol(int64_t N, int64_t batch, const double* c, double* chat, double eps, hipStream_t stream);
int cheb_eval_leggrid_tol(int64_t N, int64_t batch, const double* chat, double* f, double eps, hipStream_t stream);
int dlt_forward_tol(int64_t N, int64_t batch, const double* c, double* f, double eps, hipStream_t stream);
int dlt_inverse_tol(int64_t N, int64_t batch, const double* f, double* c, double eps, hipStream_t stream);
int cheb2leg_tol(int64_t N, int64_t batch, const double* chat, double* c, double eps, hipStream_t stream);

/* cheb_eval_leggrid (eq. (3)), dlt_forward (eq. (1)) and dlt_inverse (eq.
 * (2), through eq. (10): the transposed evaluation y = T^T D_w f about the
 * grid) with the Taylor series of Sec. 2.3 taken about another equispaced
 * grid, chosen by `grid`:
 *   DLT_GRID_CHEB1     theta^cheb1_k = (k+1/2) pi/N: the same calls as the
 *                      plain entry points;
 *   DLT_GRID_CHEBSTAR  theta^cheb*_k = (k+3/4) pi/(N+1/2), the zeros of the
 *                      leading term of the Stieltjes asymptotic form (Sec. 2.2).
 *                      The nodes lie within 1/(6 pi N) of them (Lemma 2), so
 *                      8 Taylor terms meet the FP64 budget (Cor. 2, second
 *                      bound) against 16 about theta^cheb1; but the sums of
 *                      each term are odd outputs of transforms of length
 *                      2N+1 (Remark 1), computed as chirp-z transforms
 *                      (cyclic convolutions of length 2N): three passes over
 *                      8 slabs of 2N complex values, about 1050 N bytes of
 *                      intermediates against about 280 N for the Taylor
 *                      passes about theta^cheb1.
 * FP64 arithmetic; accuracy as stated at the top of this file.  N must be a
 * power of two for DLT_GRID_CHEBSTAR (DLT_ERR_UNSUPPORTED otherwise); other
 * values of grid give DLT_ERR_INVALID_ARG; arguments, layout and ownership as
 * for the plain entry points.  DLT_GRID_CHEBSTAR calls run every kernel
 * directly on `stream` (no side streams, no graph capture); the first call
 * for a size builds its tables (and the size's FP64 plan if needed) and
 * synchronises the device; the stream's workspace grows by 8 x 2N complex
 * values per instance (batches beyond the workspace bound run in slices). */
#define DLT_GRID_CHEB1 0
#define DLT_GRID_CHEBSTAR 1
int cheb_eval_leggrid_grid(int64_t N, int64_t batch, const double* chat, double* f, int grid, hipStream_t stream);
int dlt_forward_grid(int64_t N, int64_t batch, const double* c, double* f, int grid, hipStream_t stream);
int dlt_inverse_grid(int64_t N, int64_t batch, const double* f, double* c, int grid, hipStream_t stream);

/* Ragged batch: `count` independent transforms of uneven sizes in one call
 * (many transforms of different N, forward and inverse mixed).
 *   Ns[i]       size of instance i (1 <= Ns[i] <= DLT_MAX_N), host array
 *   offsets[i]  element offset of instance i in `in` and in `out` (host array;
 *               instance i reads in[offsets[i] .. offsets[i]+Ns[i]) and writes
 *               out[offsets[i] .. offsets[i]+Ns[i]))
 *   inverse[i]  0: DLT (eq. (1)), 1: IDLT (eq. (2)); host array, NULL = all 0
 *   in, out     device arrays; the spans they cover must not overlap
 *   prec        DLT_PREC_* as for the _ex entry points
 * Instances are grouped by direction and padded power-of-two size; each group
 * runs as one batched pipeline (in slices bounded by the workspace).  The
 * first call with a given descriptor (count, Ns, offsets, inverse, prec, in,
 * out, stream) times the candidate grid sizes of each group (autotuner, once
 * per group shape), builds the device descriptors and captures the whole
 * sequence into a HIP graph; it synchronises the device.  Later calls with the
 * same descriptor launch the cached graph on `stream` and do not
 * synchronise; while the kernel trace is on they run its kernels directly
 * on `stream` instead, each traced.  Graphs, descriptors and their workspaces live until
 * dlt_release(), or until a new descriptor would bring the cached graphs
 * beyond 64 or their workspaces beyond 16 GiB: that call then synchronises
 * the device and drops the cached ones. */
int dlt_batch_ex(int64_t count, const int64_t* Ns, const int64_t* offsets, const int8_t* inverse,
                 const double* in, double* out, int prec, hipStream_t stream);

/* The grid size on which dlt_batch_ex runs instances of size N in direction
 * `inverse` (0: DLT, 1: IDLT) and precision mode prec (DLT_PREC_*) on the
 * current device: the padded power of two P >= N, or 2P when the timing of
 * both at the first dlt_batch_ex call holding such instances found 2P faster
 * (on the finer grid the nodes lie closer to grid points, so the evaluation
 * needs fewer Taylor terms, which can outweigh the larger FFTs).
 * Writes it to *grid: P when 2P > DLT_MAX_N (no other candidate), 0 when no
 * dlt_batch_ex call on this device has held such instances since the last
 * dlt_release().  Host-side lookup only: no device work, no allocation, no
 * synchronisation.  Status: DLT_ERR_INVALID_ARG (N < 1, inverse not 0 or 1,
 * grid NULL, prec not a DLT_PREC_* value), DLT_ERR_UNSUPPORTED (N >
 * DLT_MAX_N). */
int dlt_batch_grid(int64_t N, int inverse, int prec, int64_t* grid);

/* dlt_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * The same transform and kernels as dlt_forward (the same bits), but the call
 * allocates nothing: every buffer beyond c and f lives in one static device
 * array of the library (32 MiB per GPU, held until the process ends), it
 * creates no stream, event or graph and never synchronises; all kernels run
 * in order on `stream`, so the call may be captured into the caller's graph.
 *   N      a power of two, 1 <= N <= 65536 (DLT_ERR_UNSUPPORTED otherwise)
 *   c, f   device arrays of N*batch doubles, as for dlt_forward; batches
 *          larger than the scratch holds run in slices inside the call
 * The plan of size N must exist beforehand: any FP64 call of size N (for
 * example dlt_forward, or dlt_plan_query(N, ...)) builds it, and that call
 * may allocate; otherwise DLT_ERR_NOT_PREPARED.  Every call on one GPU uses
 * that GPU's one scratch array: calls that may overlap in time on that GPU
 * (different streams with no ordering between them) race and give wrong
 * results; order them on one stream.  The kernel trace does not record these
 * calls. */
int dlt_forward_noalloc(int64_t N, int64_t batch, const double* c, double* f, hipStream_t stream);

/* Human-readable text of a status code (static storage). */
const char* dlt_status_string(int status);

/* Plan parameters for size N (creates the plan if needed).  Writes up to
 * max_fields of: L (Taylor terms), nd (dense columns), far-field terms,
 * far-field blocks, max terms per block, near-field chunk items, near rows
 * per end, N1, N2, pass-A tile columns, pass-B tile rows, pass-B term groups,
 * transposed-near work-groups, transposed-near row groups, near-field
 * recurrence steps (rows x degrees, one end), boundary nodes, workspace bytes
 * per instance, near-field steps that carry weights (rows x degrees >= nd),
 * pass-A term groups, and the per-stream workspace bound in bytes (a batch
 * whose workspace, instances x bytes per instance, exceeds it runs in the
 * fewest slices of at most floor(bound / bytes per instance) instances, of
 * equal size up to one instance), and the Taylor terms of the evaluation
 * about theta^cheb* (DLT_GRID_CHEBSTAR; FP64 plans of the fixed budget, 0
 * for the others).  Returns the number of fields available or a status < 0. */
int dlt_plan_query(int64_t N, int64_t* out, int max_fields);
/* The same for the plan of precision mode `prec` (DLT_PREC_*). */
int dlt_plan_query_ex(int64_t N, int prec, int64_t* out, int max_fields);
/* The same for the plan of working tolerance eps (see the _tol entry points). */
int dlt_plan_query_tol(int64_t N, double eps, int64_t* out, int max_fields);

/* Kernel trace.  While enabled, every kernel the library launches in a
 * transform is given a start and an end hipEvent bound to its own dispatch
 * (hipExtLaunchKernel; no host synchronisation at launch time), so the time
 * between them is the kernel's execution, without the dispatch around it
 * (plan set-up kernels are not traced).  dlt_trace_collect waits for the
 * events, writes at most max_kernels entries -- kernel name (NUL-terminated,
 * truncated to name_len-1 bytes, at names + i*name_len), total milliseconds
 * and launch count, summed over launches -- clears the record and returns the
 * number of entries written (>= 0) or a negative status.  While the trace
 * is on, calls run every kernel on the caller's stream alone (no side
 * streams), so a traced duration is the kernel's own and not time shared
 * with concurrent kernels; a traced call is therefore slower than an
 * untraced one.  Intended for measurement runs; tracing is off by default. */
int dlt_trace_enable(int on);
int dlt_trace_collect(int max_kernels, char* names, int name_len, double* total_ms, int64_t* counts);

/* Frees every cached plan and workspace (device memory).  Waits for the
 * device to finish; the library may be used again afterwards. */
int dlt_release(void);

#ifdef __cplusplus
}
#endif

#endif /* DLT_H_ */
