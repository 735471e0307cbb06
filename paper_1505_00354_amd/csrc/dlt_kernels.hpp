// Host-side launchers for the DLT pipelines (implemented with the kernels).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "dlt_plan.hpp"

namespace dlt {

// Device scratch for `nb` instances of one plan, carved from one buffer.
struct Work {
    cplx* X;          // far-field / DCT / Taylor DFT intermediates
    double* v;        // far-field partial values (tgB slabs)
    double* items;    // near-field (even, odd) degree sums per (row, chunk)
    double* near;     // near-field values of the endpoint rows
    double* dense;    // dense-block partials (+ reduced slab at the end)
    double* chat;     // Chebyshev coefficients
    double* vec;      // spare length-N vector
    double* part;     // near-field per-row-group sums over degrees (inverse)
    char* sub;        // scratch of the low-degree sub-run (nb instances of the sub-plan)
    int64_t sX, sv, sitems, snear, sdense, schat, svec, spart;  // per-instance strides (elements)
};

// Streams of one call: work is enqueued on `s`; independent parts may go to
// the side streams (default priority) and are joined back through events.
// With no side streams everything runs on `s`.
constexpr int LANE_SIDES = 3;
constexpr int LANE_EVENTS = 18;
// largest size whose inverse runs its nested transposed conversion's low
// block on a side stream of its own
constexpr int64_t NESTED_LOW_MAX_N = int64_t(1) << 18;
// largest size whose transposed near field runs on a side stream beside the
// transposed far field (larger sizes run it in sequence)
constexpr int64_t TNEAR_SIDE_MAX_N = int64_t(1) << 18;
struct Lanes {
    hipStream_t s = nullptr;
    hipStream_t side[LANE_SIDES] = {};
    hipEvent_t ev[LANE_EVENTS] = {};
    // the near field goes on side[2] directly, after work already ordered
    // there (no fork from s)
    bool near_inline = false;
    // the low block goes on side[1] directly: the caller of a nested run
    // forked that stream from its own stream (so no side stream waits on
    // another that also waits on it)
    bool low_inline = false;
    hipStream_t aux(int i) const { return side[i] ? side[i] : s; }
    // the same call on one stream only (used for nested runs)
    Lanes on(hipStream_t st) const {
        Lanes l;
        l.s = st;
        return l;
    }
    // the low-degree conversion nested in a Legendre-to-Chebyshev run: its
    // own work on st, its near field queued on this run's near-field stream
    // behind this run's near field (events 14, 15 are reserved for it)
    Lanes nested_leg2cheb(hipStream_t st) const {
        if (!side[2] || !ev[14]) return on(st);
        Lanes l;
        l.s = st;
        l.side[2] = side[2];
        l.near_inline = true;
        l.ev[4] = ev[14];
        l.ev[14] = ev[15];
        return l;
    }
    // the transposed conversion nested in the inverse's: its low block on
    // this run's first side stream (forked by the caller with event 16,
    // joined into st with event 17), the rest on st
    Lanes nested_leg2cheb_t(hipStream_t st) const {
        Lanes l;
        l.s = st;
        if (side[0] && ev[16] && ev[17]) {
            l.side[1] = side[0];
            l.low_inline = true;
            l.ev[9] = ev[17];
        }
        return l;
    }
};
size_t work_bytes(const Plan& p, int64_t nb);
void work_carve(const Plan& p, int64_t nb, void* base, Work& w);

// theta, w, dtheta (any may be null) for the plan's N
hipError_t run_nodes(const Plan& p, double* theta, double* w, double* dth, const Lanes& L);
// Input-independent plan data formed on the device once per plan (and its
// sub-plans): the far-field amplitude and row-factor tables and the
// near-field states at every chunk start.  Synchronous.
hipError_t plan_prepare(Plan& p);
// chat = M c for nb instances (batch strides cs, hs in elements)
hipError_t run_leg2cheb(const Plan& p, int64_t nb, const double* c, int64_t cs, double* chat, int64_t hs, Work& w,
                        const Lanes& L);
// chat_n = (eps_n/N) sum_j v_j cos(n theta_j), theta_j = (j+1/2) pi/N: the
// Chebyshev coefficients of the interpolant of values v on the grid (the
// conversion's DCT-II passes alone)
hipError_t run_chebvals2cheb(const Plan& p, int64_t nb, const double* v, int64_t vs, double* chat, int64_t hs,
                             Work& w, const Lanes& L);
// x[0..n) = 0 on stream s
hipError_t run_fill_zero(double* x, int64_t n, hipStream_t s);
// out = M^T y (times n + 1/2 when half != 0)
hipError_t run_leg2cheb_t(const Plan& p, int64_t nb, const double* y, int64_t ys, double* out, int64_t os, int half,
                          Work& w, const Lanes& L);
// f = sum_n chat_n cos(n theta^leg), dth = theta^leg - theta^cheb1.  With
// per-row tables `rr` (ragged batch) the nodes come from rr, outputs go to
// f + rr->offs[b] and dth is unused; Q > 0 overrides the plan's Taylor pairs.
hipError_t run_ndct(const Plan& p, int64_t nb, const double* chat, int64_t hs, const double* dth, double* f,
                    Work& w, const Lanes& L, const RaggedRows* rr = nullptr, int Q = 0);

// theta^cheb* evaluation: star_prepare forms the plan's H table (allocates,
// synchronises the device); run_star evaluates nb expansions chat (stride hs)
// at the Legendre nodes (dth: offsets from theta^cheb1) into f (stride fs),
// or, given the weights wts, the transposed evaluation y_n = sum_k wts_k
// in_k T_n(x_k) of in = chat into f; on stream s only, with X holding
// nb x L slabs of 2N complex values.
hipError_t star_prepare(StarPlan& sp);
hipError_t run_star(const StarPlan& sp, int64_t nb, const double* chat, int64_t hs, const double* wts,
                    const double* dth, double* f, int64_t fs, cplx* X, hipStream_t s);

// c = D_s M^T T^T D_w f (inverse transform), wts/dth from the nodes; with
// `rr` the inputs are f + rr->offs[b] paired through rr (wts, dth unused) and
// c has stride p.N.
hipError_t run_inverse(const Plan& p, int64_t nb, const double* f, const double* wts, const double* dth,
                       double* c, Work& w, const Lanes& L, const RaggedRows* rr = nullptr, int Q = 0);

// Ragged batches: node tables on the grid of size Ng for nb instances
// (R, ioff, boff device arrays; totals of interior and boundary nodes), and
// the zero-padded gather / scatter between the caller's layout and the grid.
// grids up to this size compute boundary nodes one thread per node
constexpr int RNODE_THREAD_MAX_NG = 1024;
// interior-node ranges of the instances start at multiples of this
constexpr int RNODE_INTERIOR_ALIGN = 64;
struct RaggedNodes {
    const RNode* R;
    const int* ioff;
    const int* boff;
    int nb, ni_total, nbnd_total;
};
hipError_t run_rnodes(const RaggedNodes& rn, int Ng, int* gk, double* dg, double* wg, double* theta, double* w,
                      double* dth, hipStream_t s);
hipError_t run_rgather(const double* in, const RNode* R, const int64_t* offs, int nb, int Ng, int64_t stride,
                       double* out, hipStream_t s);
hipError_t run_rscatter(const double* in, int64_t stride, const RNode* R, const int64_t* offs, int nb, int Ng,
                        double* out, hipStream_t s);

// kernel trace (start and end events bound to every traced launch)
bool trace_on();
void trace_set(bool enable);
// while held (this thread), launches are never traced (no trace events are
// created or recorded)
void trace_hold(bool hold);
int trace_collect(std::vector<std::pair<std::string, std::pair<double, int64_t>>>& out);

}  // namespace dlt
