// C ABI: argument validation, plan and workspace caches, and the order in
// which the pipelines are enqueued.  Declared in include/dlt.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/dlt.h"
#include "dlt_kernels.hpp"

using namespace dlt;

namespace {

// Device arrays describing nb instances: node parameters, offsets in the
// caller's arrays, prefix sums of interior and boundary node counts.
struct RDesc {
    RNode* R = nullptr;
    int64_t* offs = nullptr;
    int* ioff = nullptr;
    int* boff = nullptr;
    int nb = 0, ni = 0, nbd = 0;
    // the node tables of the slice (grid row -> node, its offset and weight),
    // input-independent: formed once when the slice is built, if small enough
    // (null: formed in the workspace by every run)
    int* gk = nullptr;
    double* dg = nullptr;
    double* wg = nullptr;
    ~RDesc() {
        void* q[] = {R, offs, ioff, boff, gk, dg, wg};
        for (void* x : q)
            if (x) (void)hipFree(x);
    }
};

// One slice of a ragged batch: instances of one direction on one grid.
struct RSlice {
    int dir = 0;  // 0: forward DLT, 1: inverse DLT, 2: leg2cheb, 3: Chebyshev evaluation, 4: nodes
    int64_t Ng = 0;
    int Q = 0;
    Plan* plan = nullptr;
    std::unique_ptr<RDesc> d;
};

struct BatchEntry {
    std::vector<RSlice> slices;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    size_t tab_bytes = 0;  // node tables held by the slices
    hipGraphExec_t exec = nullptr;
    ~BatchEntry() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (ws) (void)hipFree(ws);
    }
};

struct SingleEntry {
    std::vector<RSlice> slices;
    size_t ws_bytes = 0;
    size_t tab_bytes = 0;
};

struct Cache {
    std::mutex mu;
    // (device, N, precision), or (device, N, TOL_KEY + tolerance step) for
    // the plans of a working tolerance
    std::map<std::tuple<int, int64_t, int>, std::unique_ptr<Plan>> plans;
    struct WS {
        void* ptr = nullptr;
        size_t bytes = 0;
    };
    std::map<std::pair<int, hipStream_t>, WS> ws;  // (device, stream)
    std::map<std::pair<int, hipStream_t>, Lanes> lanes;  // (device, stream): side streams, events
    std::map<int64_t, RNode> rnodes;                     // host node parameters per N
    std::map<std::pair<int, hipStream_t>, hipStream_t> capture;  // (device, stream) -> private capture stream
    // equal-size batches of a size that is not a power of two: (device, N, batch, direction, precision)
    std::map<std::tuple<int, int64_t, int64_t, int, int>, std::unique_ptr<SingleEntry>> single;
    std::map<std::vector<int64_t>, std::unique_ptr<BatchEntry>> graphs;  // descriptor -> graph
    std::map<std::tuple<int, int, int64_t, int>, int64_t> tuned;  // (device, direction, P, prec) -> grid
    // repeated single calls: (device, operation, N, batch, plan, input,
    // output, stream) -> graph of the call, and the workspace it was captured with
    struct CallGraph {
        hipGraphExec_t exec = nullptr;
        void* ws = nullptr;
        int seen = 0;
    };
    std::map<std::tuple<int, int, int64_t, int64_t, const void*, const void*, void*, hipStream_t>, CallGraph> calls;
};

Cache& cache() {
    static Cache* c = new Cache();  // never destroyed: device memory goes with the process
    return *c;
}

const size_t WS_CAP = size_t(6) << 30;  // per-stream workspace bound; larger batches run in slices
// ragged-batch graphs kept at once, and the bound on their workspaces' sum
constexpr size_t BATCH_GRAPHS_MAX = 64;
const size_t BATCH_WS_MAX = size_t(16) << 30;
// Taylor pairs of cheb_eval_nodes: L = 20 gives (pi/2)^20 / 20! = 3.4e-15, within
// the FP64 Taylor budget for offsets |N dtheta| <= pi/2 (the workspace holds
// RAGGED_Q_MAX pairs)
constexpr int NODES_Q = 10;
static_assert(NODES_Q <= RAGGED_Q_MAX, "workspace");

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

int check_size(int64_t N, int64_t batch) {
    if (N < 1 || batch < 0) return DLT_ERR_INVALID_ARG;
    if (N > DLT_MAX_N || !is_pow2(N)) return DLT_ERR_UNSUPPORTED;
    return DLT_OK;
}

bool overlap(const void* a, const void* b, size_t bytes) {
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bytes && y < x + bytes;
}

// [a, a + abytes) and [b, b + bbytes) intersect
bool overlap2(const void* a, size_t abytes, const void* b, size_t bbytes) {
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bbytes && y < x + abytes;
}

int check_prec(int prec) {
    return (prec == DLT_PREC_FP64 || prec == DLT_PREC_FP32_BULK || prec == DLT_PREC_FP64_RELAXED) ? DLT_OK
                                                                                                : DLT_ERR_INVALID_ARG;
}

// the plan's node arrays (theta, w, dtheta), formed once on the device
static int plan_nodes(Plan& p) {
    const size_t vb = (size_t)p.N * sizeof(double);
    if (hipMalloc(&p.d_theta, vb) != hipSuccess || hipMalloc(&p.d_w, vb) != hipSuccess ||
        hipMalloc(&p.d_dth, vb) != hipSuccess)
        return DLT_ERR_NOMEM;
    Lanes L;
    L.s = nullptr;
    if (run_nodes(p, p.d_theta, p.d_w, p.d_dth, L) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return DLT_ERR_HIP;
    return DLT_OK;
}

int get_plan(int64_t N, int prec, Plan** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DLT_ERR_HIP;
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto key = std::make_tuple(dev, N, prec);
    auto it = c.plans.find(key);
    if (it != c.plans.end()) {
        *out = it->second.get();
        return DLT_OK;
    }
    std::unique_ptr<Plan> p(new Plan());
    int rc = plan_build(N,
                        prec == DLT_PREC_FP32_BULK   ? PREC_FP32_BULK
                        : prec == DLT_PREC_FP64_RELAXED ? PREC_FP64_RELAXED
                                                        : PREC_FP64,
                        *p);
    if (rc == DLT_OK && plan_prepare(*p) != hipSuccess) rc = DLT_ERR_HIP;
    if (rc == DLT_OK) rc = plan_nodes(*p);
    if (rc != DLT_OK) {
        plan_free(*p);
        return rc;
    }
    *out = p.get();
    c.plans[key] = std::move(p);
    return DLT_OK;
}

// the plan of (current device, N, prec) if it has been built, else null
Plan* find_plan(int64_t N, int prec) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.plans.find(std::make_tuple(dev, N, prec));
    return it == c.plans.end() ? nullptr : it->second.get();
}

// Working tolerances: the steps 1, 2, 5 x 10^e from TOL_MIN to TOL_MAX; a
// requested eps is served by the largest step not above it (its accuracy is
// then at least the requested one).
constexpr double TOL_MIN = 5e-14, TOL_MAX = 1e-1;
constexpr int TOL_KEY = 1000;
int tol_step(double eps, double* val, int* index) {
    if (!(eps >= TOL_MIN && eps <= TOL_MAX)) return DLT_ERR_INVALID_ARG;  // NaN too
    int idx = -1;
    double best = 0;
    int k = 0;
    for (int e = -14; e <= -1; ++e) {
        for (double m : {1.0, 2.0, 5.0}) {
            const double v = m * std::pow(10.0, e);
            if (v < TOL_MIN * (1 - 1e-9) || v > TOL_MAX * (1 + 1e-9)) continue;
            if (v <= eps * (1 + 1e-12)) {
                best = v;
                idx = k;
            }
            ++k;
        }
    }
    if (idx < 0) return DLT_ERR_INVALID_ARG;
    *val = best;
    *index = idx;
    return DLT_OK;
}

int get_plan_tol(int64_t N, double eps, Plan** out) {
    double tv;
    int ti, rc;
    if ((rc = tol_step(eps, &tv, &ti))) return rc;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DLT_ERR_HIP;
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto key = std::make_tuple(dev, N, TOL_KEY + ti);
    auto it = c.plans.find(key);
    if (it != c.plans.end()) {
        *out = it->second.get();
        return DLT_OK;
    }
    std::unique_ptr<Plan> p(new Plan());
    rc = plan_build(N, PREC_FP64, *p, tv);
    if (rc == DLT_OK && plan_prepare(*p) != hipSuccess) rc = DLT_ERR_HIP;
    if (rc == DLT_OK) rc = plan_nodes(*p);
    if (rc != DLT_OK) {
        plan_free(*p);
        return rc;
    }
    *out = p.get();
    c.plans[key] = std::move(p);
    return DLT_OK;
}

// workspace of at least `bytes` ordered on `s`
int get_ws(hipStream_t s, size_t bytes, void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DLT_ERR_HIP;
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    Cache::WS& w = c.ws[std::make_pair(dev, s)];
    if (w.bytes < bytes) {
        if (w.ptr) {
            // earlier work on this stream may still read the old buffer
            if (hipStreamSynchronize(s) != hipSuccess) return DLT_ERR_HIP;
            if (hipFree(w.ptr) != hipSuccess) return DLT_ERR_HIP;
            w.ptr = nullptr;
            w.bytes = 0;
        }
        if (hipMalloc(&w.ptr, bytes) != hipSuccess) {
            w.ptr = nullptr;
            return DLT_ERR_NOMEM;
        }
        w.bytes = bytes;
    }
    *out = w.ptr;
    return DLT_OK;
}

// Side streams (default priority, non-blocking) and events for calls on
// stream s of the current device, created on first use.
int get_lanes(hipStream_t s, Lanes* out) {
    // with the kernel trace on every kernel runs alone on the call's stream,
    // so that each traced duration is the kernel's own, not shared time
    if (trace_on()) {
        *out = Lanes();
        out->s = s;
        return DLT_OK;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DLT_ERR_HIP;
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto key = std::make_pair(dev, s);
    auto it = c.lanes.find(key);
    if (it == c.lanes.end()) {
        Lanes l;
        for (int i = 0; i < LANE_SIDES; ++i)
            if (hipStreamCreateWithFlags(&l.side[i], hipStreamNonBlocking) != hipSuccess) return DLT_ERR_HIP;
        for (int i = 0; i < LANE_EVENTS; ++i)
            if (hipEventCreateWithFlags(&l.ev[i], hipEventDisableTiming) != hipSuccess) return DLT_ERR_HIP;
        it = c.lanes.emplace(key, l).first;
    }
    *out = it->second;
    out->s = s;
    return DLT_OK;
}

// node arrays shared by a call: [theta | w | dtheta] after the per-instance part
struct CallWS {
    Work work;
    double* theta;
    double* w;
    double* dth;
    int64_t nb;  // instances per slice
    Lanes lanes;
};

int setup_call(const Plan& p, int64_t batch, hipStream_t s, CallWS& cw) {
    size_t per = p.ws_per_inst;
    int64_t nb = batch;
    if (per > 0 && (size_t)nb * per > WS_CAP) {
        // as few slices as the bound allows, of equal size (the last one no
        // smaller than the others by more than one instance)
        const int64_t nbmax = std::max<int64_t>(1, (int64_t)(WS_CAP / per));
        const int64_t slices = (batch + nbmax - 1) / nbmax;
        nb = (batch + slices - 1) / slices;
    }
    if (batch > 0 && nb < 1) nb = 1;
    size_t shared = p.ws_shared;
    void* base = nullptr;
    int rc = get_ws(s, shared + work_bytes(p, nb), &base);
    if (rc) return rc;
    size_t vecb = ((size_t)p.N * sizeof(double) + 255) & ~size_t(255);
    cw.theta = (double*)base;
    cw.w = (double*)((char*)base + vecb);
    cw.dth = (double*)((char*)base + 2 * vecb);
    work_carve(p, nb, (char*)base + shared, cw.work);
    cw.nb = nb;
    return get_lanes(s, &cw.lanes);
}

int hip_status(hipError_t e) { return e == hipSuccess ? DLT_OK : DLT_ERR_HIP; }

int capture_stream(hipStream_t user, hipStream_t* out);

// Runs one call: enqueue(cw) puts the call's work on cw.lanes.s (forking to
// its side streams).  The first call with a given (operation, size, batch,
// precision, buffers, stream) runs directly; the second is captured into a
// HIP graph on the private capture stream (the side streams become branches
// of the graph), and it and every later call replay that graph on the
// caller's stream with one launch.  A graph is recaptured when the stream's
// workspace has moved; traced calls always run directly.
constexpr size_t CALL_GRAPHS_MAX = 256;
// DLT_CALL_GRAPHS=0 in the environment (read once) runs every call directly
bool call_graphs_on() {
    static const bool on = [] {
        const char* v = std::getenv("DLT_CALL_GRAPHS");
        return !(v && v[0] == '0' && v[1] == 0);
    }();
    return on;
}
template <class F>
int run_call(int op, const Plan& p, int64_t batch, const void* in, void* out, hipStream_t stream, F&& enqueue) {
    CallWS cw;
    int rc = setup_call(p, batch, stream, cw);
    if (rc) return rc;
    if (trace_on() || !call_graphs_on()) return enqueue(cw);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DLT_ERR_HIP;
    void* ws = (void*)cw.theta;  // base of the stream's workspace
    const auto key = std::make_tuple(dev, op, (int64_t)p.N, batch, (const void*)&p, in, out, stream);
    Cache& c = cache();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        Cache::CallGraph& g = c.calls[key];
        if (g.exec && g.ws == ws) return hip_status(hipGraphLaunch(g.exec, stream));
        if (++g.seen < 2) return enqueue(cw);
    }
    hipStream_t cs;
    if ((rc = capture_stream(stream, &cs))) return rc;
    CallWS cc = cw;
    if ((rc = get_lanes(cs, &cc.lanes))) return rc;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) return DLT_ERR_HIP;
    rc = enqueue(cc);
    const hipError_t ce = hipStreamEndCapture(cs, &graph);
    if (rc == DLT_OK && ce != hipSuccess) rc = DLT_ERR_HIP;
    if (rc == DLT_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) rc = DLT_ERR_HIP;
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        if (c.calls.size() > CALL_GRAPHS_MAX) {
            // many distinct calls: drop the graphs of the others, once the
            // device has drained (a replay may still run on another stream)
            if (hipDeviceSynchronize() != hipSuccess) {
                (void)hipGraphExecDestroy(exec);
                return DLT_ERR_HIP;
            }
            for (auto& kv : c.calls)
                if (kv.second.exec && kv.first != key) (void)hipGraphExecDestroy(kv.second.exec);
            Cache::CallGraph mine = c.calls[key];
            c.calls.clear();
            c.calls[key] = mine;
        }
        Cache::CallGraph& g = c.calls[key];
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g.exec = exec;
        g.ws = ws;
    }
    return hip_status(hipGraphLaunch(exec, stream));
}

// ------------------------------------------------------------ ragged sizes --
// Sizes that are not powers of two, and batches of uneven sizes, run on the
// power-of-two grid Ng >= N of the Chebyshev points (j+1/2) pi/Ng: inputs are
// zero-padded to Ng (the Legendre-to-Chebyshev map and the DCTs are exact on
// the finer grid), and every Legendre node is paired with its nearest grid
// row (the Taylor series then runs with |Ng dtheta| <= pi/2, so more terms).

int64_t next_pow2(int64_t n) {
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Taylor pairs for sizes Ns on the grid Ng: the smallest L with
// r^L / L! <= tol, r = max over the sizes of |Ng dtheta| * N/Ng (<= 0.83845
// when N = Ng, Lemma 2; <= (pi/2) N/Ng otherwise).
int ragged_Q(int prec, const int64_t* Ns, const std::vector<int64_t>& idx, int64_t Ng) {
    double r = 0;
    for (int64_t i : idx)
        r = std::max(r, Ns[i] == Ng ? 0.83845 : 1.5707963267948966 * (double)Ns[i] / (double)Ng);
    const double tol = (prec == DLT_PREC_FP64) ? 5e-15 : 5e-7;
    int L = 1;
    double f = r;
    while (f > tol && L < 64) {
        ++L;
        f *= r / L;
    }
    return std::max(1, (L + 1) / 2);
}

// node parameters of size N (host, cached; caller holds the cache lock)
const RNode& rnode_of(Cache& c, int64_t N) {
    auto it = c.rnodes.find(N);
    if (it == c.rnodes.end()) {
        RNode r;
        rnode_build(N, r);
        it = c.rnodes.emplace(N, r).first;
    }
    return it->second;
}

// Builds the device descriptor of instances idx (sizes Ns, offsets offs).
// Synchronous (host-to-device copies).
int rdesc_build(const int64_t* Ns, const int64_t* offs, const std::vector<int64_t>& idx, RDesc& d) {
    const int nb = (int)idx.size();
    std::vector<RNode> R(nb);
    std::vector<int64_t> o(nb);
    std::vector<int> io(nb + 1, 0), bo(nb + 1, 0);
    {
        Cache& c = cache();
        std::lock_guard<std::mutex> lk(c.mu);
        for (int b = 0; b < nb; ++b) {
            R[b] = rnode_of(c, Ns[idx[b]]);
            o[b] = offs[idx[b]];
            const int nh = (int)((Ns[idx[b]] + 1) / 2);
            const int ni = nh - R[b].P.kb;  // rounded up: a wave serves one instance
            io[b + 1] = io[b] + (ni + RNODE_INTERIOR_ALIGN - 1) / RNODE_INTERIOR_ALIGN * RNODE_INTERIOR_ALIGN;
            bo[b + 1] = bo[b] + R[b].P.kb;
        }
    }
    d.nb = nb;
    d.ni = io[nb];
    d.nbd = bo[nb];
    auto up = [](const void* h, size_t bytes, void** dst) {
        if (hipMalloc(dst, bytes) != hipSuccess) return DLT_ERR_NOMEM;
        return hipMemcpy(*dst, h, bytes, hipMemcpyHostToDevice) == hipSuccess ? DLT_OK : DLT_ERR_HIP;
    };
    int rc;
    if ((rc = up(R.data(), R.size() * sizeof(RNode), (void**)&d.R))) return rc;
    if ((rc = up(o.data(), o.size() * sizeof(int64_t), (void**)&d.offs))) return rc;
    if ((rc = up(io.data(), io.size() * sizeof(int), (void**)&d.ioff))) return rc;
    return up(bo.data(), bo.size() * sizeof(int), (void**)&d.boff);
}

size_t al256z(size_t x) { return (x + 255) & ~size_t(255); }

// workspace of a slice: the plan's per-instance work, the staging vectors
// and the node tables on the grid
size_t rslice_bytes(const Plan& p, int64_t nb) {
    const size_t v = (size_t)nb * (size_t)p.N;
    return work_bytes(p, nb) + al256z(v * sizeof(double)) + al256z(v * sizeof(int)) + 2 * al256z(v * sizeof(double));
}

// Enqueues slice S (in/out: the caller's arrays, indexed through the offsets).
hipError_t rslice_run(const RSlice& S, const double* in, double* out, void* ws, const Lanes& L) {
    const Plan& p = *S.plan;
    const int nb = S.d->nb, Ng = (int)S.Ng;
    Work w;
    work_carve(p, nb, ws, w);
    char* q = (char*)ws + work_bytes(p, nb);
    const size_t v = (size_t)nb * (size_t)Ng;
    double* stage = (double*)q;
    q += al256z(v * sizeof(double));
    int* gk = (int*)q;
    q += al256z(v * sizeof(int));
    double* dg = (double*)q;
    q += al256z(v * sizeof(double));
    double* wg = (double*)q;
    const RaggedNodes rn{S.d->R, S.d->ioff, S.d->boff, nb, S.d->ni, S.d->nbd};
    const bool cached = S.d->gk != nullptr;  // the slice's own node tables
    if (cached) {
        gk = S.d->gk;
        dg = S.d->dg;
        wg = S.d->wg;
    }
    const RaggedRows rr{gk, dg, wg, S.d->offs};
    hipError_t e;
    if (S.dir == 0) {
        if (cached) {
            if ((e = run_rgather(in, S.d->R, S.d->offs, nb, Ng, Ng, stage, L.s)) != hipSuccess) return e;
            if ((e = run_leg2cheb(p, nb, stage, Ng, w.chat, w.schat, w, L)) != hipSuccess) return e;
            return run_ndct(p, nb, w.chat, w.schat, nullptr, out, w, L, &rr, S.Q);
        }
        // nodes on the first side stream, beside the conversion
        const hipStream_t sn = L.aux(0);
        if (sn != L.s) {
            if ((e = hipEventRecord(L.ev[12], L.s)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(sn, L.ev[12], 0)) != hipSuccess) return e;
        }
        if ((e = run_rnodes(rn, Ng, gk, dg, nullptr, nullptr, nullptr, nullptr, sn)) != hipSuccess) return e;
        if (sn != L.s && (e = hipEventRecord(L.ev[13], sn)) != hipSuccess) return e;
        if ((e = run_rgather(in, S.d->R, S.d->offs, nb, Ng, Ng, stage, L.s)) != hipSuccess) return e;
        if ((e = run_leg2cheb(p, nb, stage, Ng, w.chat, w.schat, w, L)) != hipSuccess) return e;
        if (sn != L.s && (e = hipStreamWaitEvent(L.s, L.ev[13], 0)) != hipSuccess) return e;
        return run_ndct(p, nb, w.chat, w.schat, nullptr, out, w, L, &rr, S.Q);
    }
    if (S.dir == 2) {  // Legendre-to-Chebyshev coefficients, the first N_b of each
        if ((e = run_rgather(in, S.d->R, S.d->offs, nb, Ng, Ng, stage, L.s)) != hipSuccess) return e;
        if ((e = run_leg2cheb(p, nb, stage, Ng, w.chat, w.schat, w, L)) != hipSuccess) return e;
        return run_rscatter(w.chat, w.schat, S.d->R, S.d->offs, nb, Ng, out, L.s);
    }
    if (S.dir == 3) {  // Chebyshev expansion (zero-padded) at the Legendre nodes
        if (!cached && (e = run_rnodes(rn, Ng, gk, dg, nullptr, nullptr, nullptr, nullptr, L.s)) != hipSuccess)
            return e;
        if ((e = run_rgather(in, S.d->R, S.d->offs, nb, Ng, Ng, stage, L.s)) != hipSuccess) return e;
        return run_ndct(p, nb, stage, Ng, nullptr, out, w, L, &rr, S.Q);
    }
    if (!cached && (e = run_rnodes(rn, Ng, gk, dg, wg, nullptr, nullptr, nullptr, L.s)) != hipSuccess) return e;
    if ((e = run_inverse(p, nb, in, nullptr, nullptr, stage, w, L, &rr, S.Q)) != hipSuccess) return e;
    return run_rscatter(stage, Ng, S.d->R, S.d->offs, nb, Ng, out, L.s);
}

// The node tables of a slice of the evaluating directions (0, 1, 3), formed
// once on the device (the null stream, then a device synchronisation: slices
// are built by first calls, which synchronise anyway) while the batch's
// tables (running total *held) stay within `cap` bytes; the slices beyond
// form them in every run.  A cached batch holds at most RTABLE_MAX bytes of
// tables, the cached equal-size batches together at most SINGLE_TABLES_MAX.
constexpr size_t RTABLE_MAX = size_t(1) << 30;
constexpr size_t SINGLE_TABLES_MAX = size_t(4) << 30;
int rdesc_tables(RSlice& S, size_t* held, size_t cap) {
    if (S.dir != 0 && S.dir != 1 && S.dir != 3) return DLT_OK;
    RDesc& d = *S.d;
    const size_t v = (size_t)d.nb * (size_t)S.Ng;
    const bool inv = S.dir == 1;
    const size_t need = v * (sizeof(int) + sizeof(double) * (inv ? 2 : 1));
    if (*held + need > cap) return DLT_OK;
    *held += need;
    if (hipMalloc(&d.gk, v * sizeof(int)) != hipSuccess || hipMalloc(&d.dg, v * sizeof(double)) != hipSuccess ||
        (inv && hipMalloc(&d.wg, v * sizeof(double)) != hipSuccess))
        return DLT_ERR_NOMEM;
    const RaggedNodes rn{d.R, d.ioff, d.boff, d.nb, d.ni, d.nbd};
    if (run_rnodes(rn, (int)S.Ng, d.gk, d.dg, d.wg, nullptr, nullptr, nullptr, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
        return DLT_ERR_HIP;
    return DLT_OK;
}

// Splits instances idx (one direction, one grid) into slices whose
// workspace fits WS_CAP; builds their descriptors (and node tables while
// *tab, to which their bytes are added, stays within tab_cap).
int rslices_build(int dir, int64_t Ng, int prec, const int64_t* Ns, const int64_t* offs,
                  const std::vector<int64_t>& idx, std::vector<RSlice>& out, size_t* ws_max, size_t* tab,
                  size_t tab_cap) {
    Plan* p;
    int rc;
    if ((rc = get_plan(Ng, prec, &p))) return rc;
    int64_t per = std::max<int64_t>(1, (int64_t)(WS_CAP / std::max<size_t>(1, rslice_bytes(*p, 1))));
    per = std::min<int64_t>(per, 32768);  // grid y limit of the gather kernels
    for (size_t a = 0; a < idx.size(); a += (size_t)per) {
        std::vector<int64_t> part(idx.begin() + a, idx.begin() + std::min(idx.size(), a + (size_t)per));
        RSlice S;
        S.dir = dir;
        S.Ng = Ng;
        S.plan = p;
        S.Q = ragged_Q(prec, Ns, part, Ng);
        S.d.reset(new RDesc());
        if ((rc = rdesc_build(Ns, offs, part, *S.d))) return rc;
        if ((rc = rdesc_tables(S, tab, tab_cap))) return rc;
        *ws_max = std::max(*ws_max, rslice_bytes(*p, (int64_t)part.size()));
        out.push_back(std::move(S));
    }
    return DLT_OK;
}

// Equal-size instances of a size that is not a power of two (batch
// instances at stride N): run directly on the caller's stream; the slices
// are built once per (device, size, batch, direction, precision).
int single_entry(int64_t N, int64_t batch, int dir, int prec, SingleEntry** out);

int ragged_equal(int64_t N, int64_t batch, int dir, const double* in, double* out, int prec, hipStream_t s) {
    SingleEntry* E = nullptr;
    int rc;
    if ((rc = single_entry(N, batch, dir, prec, &E))) return rc;
    void* ws = nullptr;
    if ((rc = get_ws(s, E->ws_bytes, &ws))) return rc;
    Lanes L;
    if ((rc = get_lanes(s, &L))) return rc;
    for (auto& S : E->slices)
        if ((rc = hip_status(rslice_run(S, in, out, ws, L)))) return rc;
    return DLT_OK;
}

int single_entry(int64_t N, int64_t batch, int dir, int prec, SingleEntry** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DLT_ERR_HIP;
    const auto key = std::make_tuple(dev, N, batch, dir, prec);
    SingleEntry* E = nullptr;
    {
        Cache& c = cache();
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.single.find(key);
        if (it != c.single.end()) E = it->second.get();
    }
    int rc;
    if (!E) {
        std::unique_ptr<SingleEntry> e(new SingleEntry());
        std::vector<int64_t> Ns(batch, N), offs(batch), idx(batch);
        for (int64_t b = 0; b < batch; ++b) {
            offs[b] = b * N;
            idx[b] = b;
        }
        size_t cap = 0;  // what the cached equal-size batches leave of their table bound
        {
            Cache& c = cache();
            std::lock_guard<std::mutex> lk(c.mu);
            size_t used = 0;
            for (auto& kv : c.single) used += kv.second->tab_bytes;
            if (used < SINGLE_TABLES_MAX) cap = std::min(RTABLE_MAX, SINGLE_TABLES_MAX - used);
        }
        if ((rc = rslices_build(dir, next_pow2(N), prec, Ns.data(), offs.data(), idx, e->slices, &e->ws_bytes,
                                &e->tab_bytes, cap)))
            return rc;
        Cache& c = cache();
        std::lock_guard<std::mutex> lk(c.mu);
        E = c.single.emplace(key, std::move(e)).first->second.get();
    }
    *out = E;
    return DLT_OK;
}

// Private stream on which batch graphs are captured (one per device and
// caller stream; capture cannot run on the legacy default stream).
int capture_stream(hipStream_t user, hipStream_t* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DLT_ERR_HIP;
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto key = std::make_pair(dev, user);
    auto it = c.capture.find(key);
    if (it == c.capture.end()) {
        hipStream_t cs = nullptr;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return DLT_ERR_HIP;
        it = c.capture.emplace(key, cs).first;
    }
    *out = it->second;
    return DLT_OK;
}

// Autotuner: for the instances idx of one direction with largest padded
// size P, time the grid Ng = P against Ng = 2P (fewer Taylor terms on a
// twice larger grid) on up to 64 of them (inputs copied to a compact
// scratch layout, outputs to scratch), once per (device, direction, P,
// precision).  Synchronous; runs before any capture.
int tune_grid(int dir, int64_t P, int prec, const int64_t* Ns, const int64_t* offs,
              const std::vector<int64_t>& idx, const double* in, hipStream_t s, int64_t* Ng) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DLT_ERR_HIP;
    const auto key = std::make_tuple(dev, dir, P, prec);
    {
        Cache& c = cache();
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.tuned.find(key);
        if (it != c.tuned.end()) {
            *Ng = it->second;
            return DLT_OK;
        }
    }
    *Ng = P;
    if (2 * P > DLT_MAX_N) return DLT_OK;
    // compact copy of a sample of the instances
    std::vector<int64_t> sub(idx.begin(), idx.begin() + std::min<size_t>(idx.size(), 64));
    std::vector<int64_t> sN(sub.size()), so(sub.size()), sidx(sub.size());
    int64_t tot = 0;
    for (size_t i = 0; i < sub.size(); ++i) {
        sN[i] = Ns[sub[i]];
        so[i] = tot;
        sidx[i] = (int64_t)i;
        tot += sN[i];
    }
    double *din = nullptr, *dout = nullptr;
    if (hipMalloc(&din, tot * sizeof(double)) != hipSuccess) return DLT_ERR_NOMEM;
    if (hipMalloc(&dout, tot * sizeof(double)) != hipSuccess) {
        (void)hipFree(din);
        return DLT_ERR_NOMEM;
    }
    int rc = DLT_OK;
    for (size_t i = 0; i < sub.size() && rc == DLT_OK; ++i)
        if (hipMemcpyAsync(din + so[i], in + offs[sub[i]], sN[i] * sizeof(double), hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
            rc = DLT_ERR_HIP;
    Lanes L;
    if (rc == DLT_OK) rc = get_lanes(s, &L);
    float best = 1e30f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == DLT_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = DLT_ERR_HIP;
    for (int64_t cand = P; cand <= 2 * P && rc == DLT_OK; cand *= 2) {
        std::vector<RSlice> sl;
        size_t wmax = 0, tab = 0;
        if ((rc = rslices_build(dir, cand, prec, sN.data(), so.data(), sidx, sl, &wmax, &tab, RTABLE_MAX))) break;
        void* ws = nullptr;
        if ((rc = get_ws(s, wmax, &ws))) break;
        float ms = 0;
        for (int rep = 0; rep < 3 && rc == DLT_OK; ++rep) {
            if (rep == 1 && hipEventRecord(e0, s) != hipSuccess) rc = DLT_ERR_HIP;
            for (auto& S : sl)
                if (rc == DLT_OK) rc = hip_status(rslice_run(S, din, dout, ws, L));
        }
        if (rc == DLT_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = DLT_ERR_HIP;
        if (rc == DLT_OK && ms < best) {
            best = ms;
            *Ng = cand;
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess && rc == DLT_OK) rc = DLT_ERR_HIP;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(din);
    (void)hipFree(dout);
    if (rc != DLT_OK) return rc;
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    c.tuned[key] = *Ng;
    return DLT_OK;
}

bool is_pow2_n(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

// arguments of the single-size entry points: power-of-two sizes take the
// plain path; other sizes up to DLT_MAX_N the padded-grid path
int check_any_size(int64_t N, int64_t batch) {
    if (N < 1 || batch < 0) return DLT_ERR_INVALID_ARG;
    if (N > DLT_MAX_N) return DLT_ERR_UNSUPPORTED;
    return DLT_OK;
}

// ------------------------------------------------ allocation-free forward --
// Device scratch of dlt_forward_noalloc: one array per GPU, held until the
// process ends.  In host code `scratch` only names the symbol; its device
// address (per device) comes from hipGetSymbolAddress.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(32) << 20;
constexpr int64_t NOALLOC_MAX_N = int64_t(1) << 16;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// the current device's address of `scratch` (looked up once per device)
int scratch_address(void** out) {
    static std::mutex mu;
    static std::map<int, void*> addr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DLT_ERR_HIP;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DLT_ERR_HIP;
        it = addr.emplace(dev, p).first;
    }
    *out = it->second;
    return DLT_OK;
}

}  // namespace

extern "C" {

int dlt_batch_ex(int64_t count, const int64_t* Ns, const int64_t* offsets, const int8_t* inverse,
                 const double* in, double* out, int prec, hipStream_t stream) {
    if (count < 0) return DLT_ERR_INVALID_ARG;
    if (count == 0) return DLT_OK;
    int rc;
    if ((rc = check_prec(prec))) return rc;
    if (!Ns || !offsets || !in || !out) return DLT_ERR_INVALID_ARG;
    int64_t lo = INT64_MAX, hi = 0;
    for (int64_t i = 0; i < count; ++i) {
        if (Ns[i] < 1 || offsets[i] < 0) return DLT_ERR_INVALID_ARG;
        if (Ns[i] > DLT_MAX_N) return DLT_ERR_UNSUPPORTED;
        if (inverse && inverse[i] != 0 && inverse[i] != 1) return DLT_ERR_INVALID_ARG;
        lo = std::min(lo, offsets[i]);
        hi = std::max(hi, offsets[i] + Ns[i]);
    }
    if (overlap(in + lo, out + lo, (size_t)(hi - lo) * sizeof(double))) return DLT_ERR_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DLT_ERR_HIP;
    std::vector<int64_t> key;
    key.reserve(3 * count + 6);
    key.push_back(dev);
    key.push_back(prec);
    key.push_back((int64_t)(uintptr_t)in);
    key.push_back((int64_t)(uintptr_t)out);
    key.push_back((int64_t)(uintptr_t)stream);
    key.push_back(count);
    for (int64_t i = 0; i < count; ++i) {
        key.push_back(Ns[i]);
        key.push_back(offsets[i]);
        key.push_back(inverse ? inverse[i] : 0);
    }
    // a cached batch: its graph, or with the kernel trace on its kernels
    // directly on `stream` (each traced, none on a side stream)
    // (called with the cache lock held: the lanes are taken before)
    const bool traced_run = trace_on();
    Lanes TL;
    if (traced_run && (rc = get_lanes(stream, &TL))) return rc;
    auto launch_entry = [&](BatchEntry* E) -> int {
        if (!traced_run) return hip_status(hipGraphLaunch(E->exec, stream));
        int r = DLT_OK;
        for (auto& S : E->slices)
            if (r == DLT_OK) r = hip_status(rslice_run(S, in, out, E->ws, TL));
        return r;
    };
    {
        Cache& c = cache();
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.graphs.find(key);
        if (it != c.graphs.end()) return launch_entry(it->second.get());
    }
    {
        std::unique_ptr<BatchEntry> e(new BatchEntry());
        // size classes: direction and padded size
        std::map<std::pair<int, int64_t>, std::vector<int64_t>> cls;
        for (int64_t i = 0; i < count; ++i) cls[{inverse ? (int)inverse[i] : 0, next_pow2(Ns[i])}].push_back(i);
        size_t wmax = 0;
        for (auto& kv : cls) {
            int64_t Ng = kv.first.second;
            if ((rc = tune_grid(kv.first.first, kv.first.second, prec, Ns, offsets, kv.second, in, stream, &Ng)))
                return rc;
            if ((rc = rslices_build(kv.first.first, Ng, prec, Ns, offsets, kv.second, e->slices, &wmax,
                                    &e->tab_bytes, RTABLE_MAX)))
                return rc;
        }
        {
            // each cached graph owns a workspace and node tables: beyond
            // BATCH_GRAPHS_MAX graphs or BATCH_WS_MAX bytes of them, drop the
            // cached ones (once the device has drained: a replay may still run)
            Cache& c = cache();
            std::lock_guard<std::mutex> lk(c.mu);
            size_t held = wmax + e->tab_bytes;
            for (auto& kv : c.graphs) held += kv.second->ws_bytes + kv.second->tab_bytes;
            if (!c.graphs.empty() && (c.graphs.size() >= BATCH_GRAPHS_MAX || held > BATCH_WS_MAX)) {
                if (hipDeviceSynchronize() != hipSuccess) return DLT_ERR_HIP;
                c.graphs.clear();
            }
        }
        if (hipMalloc(&e->ws, wmax) != hipSuccess) return DLT_ERR_NOMEM;
        e->ws_bytes = wmax;
        // capture every slice into one graph on a private stream
        hipStream_t cs;
        if ((rc = capture_stream(stream, &cs))) return rc;
        // the graph is cached: capture it untraced, with its side streams
        const bool tr = trace_on();
        trace_set(false);
        Lanes L;
        if ((rc = get_lanes(cs, &L))) {
            trace_set(tr);
            return rc;
        }
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) rc = DLT_ERR_HIP;
        for (auto& S : e->slices)
            if (rc == DLT_OK) rc = hip_status(rslice_run(S, in, out, e->ws, L));
        hipError_t ce = hipStreamEndCapture(cs, &g);
        trace_set(tr);
        if (rc == DLT_OK && ce != hipSuccess) rc = DLT_ERR_HIP;
        if (rc == DLT_OK && hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0) != hipSuccess) rc = DLT_ERR_HIP;
        if (g) (void)hipGraphDestroy(g);
        if (rc) return rc;
        Cache& c = cache();
        std::lock_guard<std::mutex> lk(c.mu);
        BatchEntry* E = c.graphs.emplace(key, std::move(e)).first->second.get();
        return launch_entry(E);
    }
}



const char* dlt_status_string(int st) {
    switch (st) {
        case DLT_OK: return "ok";
        case DLT_ERR_INVALID_ARG: return "invalid argument";
        case DLT_ERR_UNSUPPORTED: return "unsupported size";
        case DLT_ERR_HIP: return "HIP runtime error";
        case DLT_ERR_NOMEM: return "out of device memory";
        case DLT_ERR_NOT_PREPARED: return "plan not prepared (dlt_forward_noalloc: build the size's plan first)";
        default: return "unknown status";
    }
}

int leg_nodes_weights(int64_t N, int64_t batch, double* theta, double* w, double* dtheta, hipStream_t stream) {
    int rc = check_any_size(N, batch);
    if (rc) return rc;
    if (batch == 0 || (!theta && !w && !dtheta)) return DLT_OK;
    size_t bytes = (size_t)N * sizeof(double) * (size_t)batch;
    if ((theta && w && overlap(theta, w, bytes)) || (theta && dtheta && overlap(theta, dtheta, bytes)) ||
        (w && dtheta && overlap(w, dtheta, bytes)))
        return DLT_ERR_INVALID_ARG;
    if (!is_pow2_n(N)) {
        SingleEntry* E;
        if ((rc = single_entry(N, 1, 4, DLT_PREC_FP64, &E))) return rc;
        const RDesc& d = *E->slices[0].d;
        const RaggedNodes rn{d.R, d.ioff, d.boff, d.nb, d.ni, d.nbd};
        if ((rc = hip_status(run_rnodes(rn, 0, nullptr, nullptr, nullptr, theta, w, dtheta, stream)))) return rc;
    } else {
        Plan* p;
        if ((rc = get_plan(N, DLT_PREC_FP64, &p))) return rc;
        const size_t vb = (size_t)N * sizeof(double);
        if (theta && hipMemcpyAsync(theta, p->d_theta, vb, hipMemcpyDeviceToDevice, stream)) return DLT_ERR_HIP;
        if (w && hipMemcpyAsync(w, p->d_w, vb, hipMemcpyDeviceToDevice, stream)) return DLT_ERR_HIP;
        if (dtheta && hipMemcpyAsync(dtheta, p->d_dth, vb, hipMemcpyDeviceToDevice, stream)) return DLT_ERR_HIP;
    }
    for (int64_t b = 1; b < batch; ++b) {
        size_t vb = (size_t)N * sizeof(double);
        if (theta && hipMemcpyAsync(theta + b * N, theta, vb, hipMemcpyDeviceToDevice, stream)) return DLT_ERR_HIP;
        if (w && hipMemcpyAsync(w + b * N, w, vb, hipMemcpyDeviceToDevice, stream)) return DLT_ERR_HIP;
        if (dtheta && hipMemcpyAsync(dtheta + b * N, dtheta, vb, hipMemcpyDeviceToDevice, stream))
            return DLT_ERR_HIP;
    }
    return DLT_OK;
}

int leg2cheb(int64_t N, int64_t batch, const double* c, double* chat, hipStream_t stream) {
    return leg2cheb_ex(N, batch, c, chat, DLT_PREC_FP64, stream);
}

// leg2cheb for nb instances on plan P (any precision mode or tolerance)
static int leg2cheb_on(Plan& P, int64_t N, int64_t batch, const double* c, double* chat, hipStream_t stream) {
    Plan* p = &P;
    return run_call(2, *p, batch, c, chat, stream, [&](CallWS& cw) -> int {
        for (int64_t b0 = 0; b0 < batch; b0 += cw.nb) {
            int64_t nb = std::min(cw.nb, batch - b0);
            int r = hip_status(run_leg2cheb(*p, nb, c + b0 * N, N, chat + b0 * N, N, cw.work, cw.lanes));
            if (r) return r;
        }
        return DLT_OK;
    });
}

int leg2cheb_ex(int64_t N, int64_t batch, const double* c, double* chat, int prec, hipStream_t stream) {
    int rc = check_any_size(N, batch);
    if (rc) return rc;
    if ((rc = check_prec(prec))) return rc;
    if (batch == 0) return DLT_OK;
    if (!c || !chat || overlap(c, chat, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    if (!is_pow2_n(N)) return ragged_equal(N, batch, 2, c, chat, prec, stream);
    Plan* p;
    if ((rc = get_plan(N, prec, &p))) return rc;
    return leg2cheb_on(*p, N, batch, c, chat, stream);
}

int leg2cheb_tol(int64_t N, int64_t batch, const double* c, double* chat, double eps, hipStream_t stream) {
    int rc = check_size(N, batch);  // power-of-two sizes
    if (rc) return rc;
    double tv;
    int ti;
    if ((rc = tol_step(eps, &tv, &ti))) return rc;
    if (batch == 0) return DLT_OK;
    if (!c || !chat || overlap(c, chat, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan_tol(N, eps, &p))) return rc;
    return leg2cheb_on(*p, N, batch, c, chat, stream);
}

int cheb_eval_leggrid(int64_t N, int64_t batch, const double* chat, double* f, hipStream_t stream) {
    return cheb_eval_leggrid_ex(N, batch, chat, f, DLT_PREC_FP64, stream);
}

// cheb_eval_leggrid for nb instances on plan P (any precision mode or tolerance)
static int cheb_eval_leggrid_on(Plan& P, int64_t N, int64_t batch, const double* chat, double* f, hipStream_t stream) {
    Plan* p = &P;
    return run_call(3, *p, batch, chat, f, stream, [&](CallWS& cw) -> int {
        for (int64_t b0 = 0; b0 < batch; b0 += cw.nb) {
            int64_t nb = std::min(cw.nb, batch - b0);
            int r = hip_status(run_ndct(*p, nb, chat + b0 * N, N, p->d_dth, f + b0 * N, cw.work, cw.lanes));
            if (r) return r;
        }
        return DLT_OK;
    });
}

int cheb_eval_leggrid_ex(int64_t N, int64_t batch, const double* chat, double* f, int prec, hipStream_t stream) {
    int rc = check_any_size(N, batch);
    if (rc) return rc;
    if ((rc = check_prec(prec))) return rc;
    if (batch == 0) return DLT_OK;
    if (!chat || !f || overlap(chat, f, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    if (!is_pow2_n(N)) return ragged_equal(N, batch, 3, chat, f, prec, stream);
    Plan* p;
    if ((rc = get_plan(N, prec, &p))) return rc;
    return cheb_eval_leggrid_on(*p, N, batch, chat, f, stream);
}

int cheb_eval_leggrid_tol(int64_t N, int64_t batch, const double* chat, double* f, double eps, hipStream_t stream) {
    int rc = check_size(N, batch);  // power-of-two sizes
    if (rc) return rc;
    double tv;
    int ti;
    if ((rc = tol_step(eps, &tv, &ti))) return rc;
    if (batch == 0) return DLT_OK;
    if (!chat || !f || overlap(chat, f, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan_tol(N, eps, &p))) return rc;
    return cheb_eval_leggrid_on(*p, N, batch, chat, f, stream);
}

int dlt_forward(int64_t N, int64_t batch, const double* c, double* f, hipStream_t stream) {
    return dlt_forward_ex(N, batch, c, f, DLT_PREC_FP64, stream);
}

// dlt_forward for nb instances on plan P (any precision mode or tolerance)
static int dlt_forward_on(Plan& P, int64_t N, int64_t batch, const double* c, double* f, hipStream_t stream) {
    Plan* p = &P;
    return run_call(0, *p, batch, c, f, stream, [&](CallWS& cw) -> int {
        const Lanes& L = cw.lanes;
        for (int64_t b0 = 0; b0 < batch; b0 += cw.nb) {
            int64_t nb = std::min(cw.nb, batch - b0);
            // Chebyshev coefficients of the slice, stride N, in the workspace
            double* chat = cw.work.chat;
            int r = hip_status(run_leg2cheb(*p, nb, c + b0 * N, N, chat, cw.work.schat, cw.work, L));
            if (r) return r;
            if ((r = hip_status(run_ndct(*p, nb, chat, cw.work.schat, p->d_dth, f + b0 * N, cw.work, L)))) return r;
        }
        return DLT_OK;
    });
}

int dlt_forward_ex(int64_t N, int64_t batch, const double* c, double* f, int prec, hipStream_t stream) {
    int rc = check_any_size(N, batch);
    if (rc) return rc;
    if ((rc = check_prec(prec))) return rc;
    if (batch == 0) return DLT_OK;
    if (!c || !f || overlap(c, f, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    if (!is_pow2_n(N)) return ragged_equal(N, batch, 0, c, f, prec, stream);
    Plan* p;
    if ((rc = get_plan(N, prec, &p))) return rc;
    return dlt_forward_on(*p, N, batch, c, f, stream);
}

int dlt_forward_tol(int64_t N, int64_t batch, const double* c, double* f, double eps, hipStream_t stream) {
    int rc = check_size(N, batch);  // power-of-two sizes
    if (rc) return rc;
    double tv;
    int ti;
    if ((rc = tol_step(eps, &tv, &ti))) return rc;
    if (batch == 0) return DLT_OK;
    if (!c || !f || overlap(c, f, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan_tol(N, eps, &p))) return rc;
    return dlt_forward_on(*p, N, batch, c, f, stream);
}

// dlt_forward with every buffer beyond c and f in the library's static
// device scratch: no allocation, no side stream, no event, no graph; every
// kernel on `stream` in order.  The scratch needs no clearing (every pass
// writes what a later pass reads before it is read).
int dlt_forward_noalloc(int64_t N, int64_t batch, const double* c, double* f, hipStream_t stream) {
    int rc = check_any_size(N, batch);
    if (rc) return rc;
    if (N > NOALLOC_MAX_N || (N & (N - 1)) != 0) return DLT_ERR_UNSUPPORTED;
    if (batch == 0) return DLT_OK;
    if (!c || !f || overlap(c, f, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    Plan* p = find_plan(N, DLT_PREC_FP64);
    if (!p) return DLT_ERR_NOT_PREPARED;
    void* base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    const size_t shared = p->ws_shared;
    if (shared + p->ws_per_inst > NOALLOC_SCRATCH_BYTES) return DLT_ERR_UNSUPPORTED;
    const int64_t per_slice =
        p->ws_per_inst ? (int64_t)((NOALLOC_SCRATCH_BYTES - shared) / p->ws_per_inst) : batch;
    const int64_t nbmax = std::min<int64_t>(batch, per_slice);
    Work work;  // after the node-array region of setup_call's layout (unused: the plan holds the nodes)
    work_carve(*p, nbmax, (char*)base + shared, work);
    Lanes L;  // the caller's stream only
    L.s = stream;
    trace_hold(true);
    for (int64_t b0 = 0; rc == DLT_OK && b0 < batch; b0 += nbmax) {
        const int64_t nb = std::min(nbmax, batch - b0);
        rc = hip_status(run_leg2cheb(*p, nb, c + b0 * N, N, work.chat, work.schat, work, L));
        if (rc == DLT_OK) rc = hip_status(run_ndct(*p, nb, work.chat, work.schat, p->d_dth, f + b0 * N, work, L));
    }
    trace_hold(false);
    return rc;
}

// ------------------------------------------------------ theta^cheb* grid --
// the theta^cheb* plan of an FP64 plan (built on first use)
static int get_star(Plan* p, StarPlan** out) {
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    if (!p->star) {
        std::unique_ptr<StarPlan> s(new StarPlan());
        int rc = star_plan_build(p->N, *s);
        if (rc == DLT_OK && star_prepare(*s) != hipSuccess) rc = DLT_ERR_HIP;
        if (rc != DLT_OK) {
            star_plan_free(*s);
            return rc;
        }
        p->star = s.release();
    }
    *out = p->star;
    return DLT_OK;
}

// cheb_eval_leggrid (op 0), dlt_forward (op 1) or dlt_inverse (op 2) about
// theta^cheb*, every kernel on `stream`, in slices that keep the workspace
// within WS_CAP
static int star_call(int64_t N, int64_t batch, const double* in, double* f, int op, hipStream_t stream) {
    const bool from_leg = op == 1, inverse = op == 2;
    Plan* p;
    int rc;
    if ((rc = get_plan(N, DLT_PREC_FP64, &p))) return rc;
    StarPlan* sp;
    if ((rc = get_star(p, &sp))) return rc;
    const size_t per = sp->ws_per_inst + (op != 0 ? p->ws_per_inst : 0);
    int64_t nb = batch;
    if ((size_t)nb * per > WS_CAP) {
        const int64_t nbmax = std::max<int64_t>(1, (int64_t)(WS_CAP / per));
        const int64_t slices = (batch + nbmax - 1) / nbmax;
        nb = (batch + slices - 1) / slices;
    }
    void* base = nullptr;
    if ((rc = get_ws(stream, p->ws_shared + (size_t)nb * per, &base))) return rc;
    const size_t vecb = ((size_t)N * sizeof(double) + 255) & ~size_t(255);
    double* wts = (double*)((char*)base + vecb);  // the layout of setup_call
    double* dth = (double*)((char*)base + 2 * vecb);
    char* q = (char*)base + p->ws_shared;
    cplx* X = (cplx*)q;  // nb x L slabs of 2N values
    Work work;
    if (op != 0) work_carve(*p, nb, q + (size_t)nb * sp->ws_per_inst, work);
    Lanes L;  // the caller's stream only
    L.s = stream;
    wts = p->d_w;
    dth = p->d_dth;
    for (int64_t b0 = 0; rc == DLT_OK && b0 < batch; b0 += nb) {
        const int64_t n = std::min(nb, batch - b0);
        if (inverse) {
            // y = T^T D_w f about theta^cheb*, then c = D_s M^T y (Sec. 4)
            rc = hip_status(run_star(*sp, n, in + b0 * N, N, wts, dth, work.chat, work.schat, X, stream));
            if (rc == DLT_OK) rc = hip_status(run_leg2cheb_t(*p, n, work.chat, work.schat, f + b0 * N, N, 1, work, L));
            continue;
        }
        const double* chat = in + b0 * N;
        int64_t hs = N;
        if (from_leg) {
            rc = hip_status(run_leg2cheb(*p, n, in + b0 * N, N, work.chat, work.schat, work, L));
            chat = work.chat;
            hs = work.schat;
        }
        if (rc == DLT_OK) rc = hip_status(run_star(*sp, n, chat, hs, nullptr, dth, f + b0 * N, N, X, stream));
    }
    return rc;
}

static int grid_args(int64_t N, int64_t batch, const double* in, const double* out) {
    int rc = check_any_size(N, batch);
    if (rc) return rc;
    if (!is_pow2_n(N)) return DLT_ERR_UNSUPPORTED;
    if (batch > 0 && (!in || !out || overlap(in, out, (size_t)N * batch * sizeof(double))))
        return DLT_ERR_INVALID_ARG;
    return DLT_OK;
}

int cheb_eval_leggrid_grid(int64_t N, int64_t batch, const double* chat, double* f, int grid, hipStream_t stream) {
    if (grid == DLT_GRID_CHEB1) return cheb_eval_leggrid(N, batch, chat, f, stream);
    if (grid != DLT_GRID_CHEBSTAR) return DLT_ERR_INVALID_ARG;
    int rc = grid_args(N, batch, chat, f);
    if (rc || batch == 0) return rc;
    return star_call(N, batch, chat, f, 0, stream);
}

int dlt_forward_grid(int64_t N, int64_t batch, const double* c, double* f, int grid, hipStream_t stream) {
    if (grid == DLT_GRID_CHEB1) return dlt_forward(N, batch, c, f, stream);
    if (grid != DLT_GRID_CHEBSTAR) return DLT_ERR_INVALID_ARG;
    int rc = grid_args(N, batch, c, f);
    if (rc || batch == 0) return rc;
    return star_call(N, batch, c, f, 1, stream);
}

int dlt_inverse_grid(int64_t N, int64_t batch, const double* f, double* c, int grid, hipStream_t stream) {
    if (grid == DLT_GRID_CHEB1) return dlt_inverse(N, batch, f, c, stream);
    if (grid != DLT_GRID_CHEBSTAR) return DLT_ERR_INVALID_ARG;
    int rc = grid_args(N, batch, f, c);
    if (rc || batch == 0) return rc;
    return star_call(N, batch, f, c, 2, stream);
}

int dlt_inverse(int64_t N, int64_t batch, const double* f, double* c, hipStream_t stream) {
    return dlt_inverse_ex(N, batch, f, c, DLT_PREC_FP64, stream);
}

// dlt_inverse for nb instances on plan P (any precision mode or tolerance)
static int dlt_inverse_on(Plan& P, int64_t N, int64_t batch, const double* f, double* c, hipStream_t stream) {
    Plan* p = &P;
    return run_call(1, *p, batch, f, c, stream, [&](CallWS& cw) -> int {
        for (int64_t b0 = 0; b0 < batch; b0 += cw.nb) {
            int64_t nb = std::min(cw.nb, batch - b0);
            int r = hip_status(run_inverse(*p, nb, f + b0 * N, p->d_w, p->d_dth, c + b0 * N, cw.work, cw.lanes));
            if (r) return r;
        }
        return DLT_OK;
    });
}

int dlt_inverse_ex(int64_t N, int64_t batch, const double* f, double* c, int prec, hipStream_t stream) {
    int rc = check_any_size(N, batch);
    if (rc) return rc;
    if ((rc = check_prec(prec))) return rc;
    if (batch == 0) return DLT_OK;
    if (!f || !c || overlap(f, c, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    if (!is_pow2_n(N)) return ragged_equal(N, batch, 1, f, c, prec, stream);
    Plan* p;
    if ((rc = get_plan(N, prec, &p))) return rc;
    return dlt_inverse_on(*p, N, batch, f, c, stream);
}

int dlt_inverse_tol(int64_t N, int64_t batch, const double* f, double* c, double eps, hipStream_t stream) {
    int rc = check_size(N, batch);  // power-of-two sizes
    if (rc) return rc;
    double tv;
    int ti;
    if ((rc = tol_step(eps, &tv, &ti))) return rc;
    if (batch == 0) return DLT_OK;
    if (!f || !c || overlap(f, c, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan_tol(N, eps, &p))) return rc;
    return dlt_inverse_on(*p, N, batch, f, c, stream);
}

// Chebyshev to Legendre coefficients on plan P: the expansion's values at
// the Legendre nodes (written into c), then the inverse transform of them in
// place (its input is read only by its first pass, before c is written)
static int cheb2leg_on(Plan& P, int64_t N, int64_t batch, const double* chat, double* c, hipStream_t stream) {
    Plan* p = &P;
    return run_call(4, *p, batch, chat, c, stream, [&](CallWS& cw) -> int {
        for (int64_t b0 = 0; b0 < batch; b0 += cw.nb) {
            int64_t nb = std::min(cw.nb, batch - b0);
            int r = hip_status(run_ndct(*p, nb, chat + b0 * N, N, p->d_dth, c + b0 * N, cw.work, cw.lanes));
            if (r) return r;
            if ((r = hip_status(run_inverse(*p, nb, c + b0 * N, p->d_w, p->d_dth, c + b0 * N, cw.work, cw.lanes))))
                return r;
        }
        return DLT_OK;
    });
}

int cheb2leg(int64_t N, int64_t batch, const double* chat, double* c, hipStream_t stream) {
    return cheb2leg_ex(N, batch, chat, c, DLT_PREC_FP64, stream);
}

int cheb2leg_ex(int64_t N, int64_t batch, const double* chat, double* c, int prec, hipStream_t stream) {
    int rc = check_any_size(N, batch);
    if (rc) return rc;
    if ((rc = check_prec(prec))) return rc;
    if (batch == 0) return DLT_OK;
    if (!chat || !c || overlap(chat, c, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    if (!is_pow2_n(N)) {
        if ((rc = ragged_equal(N, batch, 3, chat, c, prec, stream))) return rc;
        return ragged_equal(N, batch, 1, c, c, prec, stream);
    }
    Plan* p;
    if ((rc = get_plan(N, prec, &p))) return rc;
    return cheb2leg_on(*p, N, batch, chat, c, stream);
}

int cheb2leg_tol(int64_t N, int64_t batch, const double* chat, double* c, double eps, hipStream_t stream) {
    int rc = check_size(N, batch);  // power-of-two sizes
    if (rc) return rc;
    double tv;
    int ti;
    if ((rc = tol_step(eps, &tv, &ti))) return rc;
    if (batch == 0) return DLT_OK;
    if (!chat || !c || overlap(chat, c, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan_tol(N, eps, &p))) return rc;
    return cheb2leg_on(*p, N, batch, chat, c, stream);
}

int cheb_eval_nodes(int64_t N, int64_t batch, const double* chat, const double* dtheta, double* f,
                    hipStream_t stream) {
    int rc = check_size(N, batch);  // power-of-two sizes
    if (rc) return rc;
    if (batch == 0) return DLT_OK;
    const size_t bytes = (size_t)N * batch * sizeof(double);
    if (!chat || !dtheta || !f || overlap(chat, f, bytes) || overlap2(dtheta, (size_t)N * sizeof(double), f, bytes))
        return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan(N, DLT_PREC_FP64, &p))) return rc;
    // enqueued directly (no cached graph: the offsets are an input of their own)
    CallWS cw;
    if ((rc = setup_call(*p, batch, stream, cw))) return rc;
    for (int64_t b0 = 0; b0 < batch; b0 += cw.nb) {
        int64_t nb = std::min(cw.nb, batch - b0);
        if ((rc = hip_status(run_ndct(*p, nb, chat + b0 * N, N, dtheta, f + b0 * N, cw.work, cw.lanes, nullptr,
                                      NODES_Q))))
            return rc;
    }
    return DLT_OK;
}

int chebvals2leg(int64_t N, int64_t batch, const double* v, double* c, hipStream_t stream) {
    int rc = check_size(N, batch);  // power-of-two sizes
    if (rc) return rc;
    if (batch == 0) return DLT_OK;
    if (!v || !c || overlap(v, c, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan(N, DLT_PREC_FP64, &p))) return rc;
    // Chebyshev coefficients of the interpolant (workspace), their expansion's
    // values at the Legendre nodes (into c), the inverse transform in place
    return run_call(5, *p, batch, v, c, stream, [&](CallWS& cw) -> int {
        for (int64_t b0 = 0; b0 < batch; b0 += cw.nb) {
            int64_t nb = std::min(cw.nb, batch - b0);
            double* chat = cw.work.chat;
            int r = hip_status(run_chebvals2cheb(*p, nb, v + b0 * N, N, chat, cw.work.schat, cw.work, cw.lanes));
            if (r) return r;
            if ((r = hip_status(run_ndct(*p, nb, chat, cw.work.schat, p->d_dth, c + b0 * N, cw.work, cw.lanes)))) return r;
            if ((r = hip_status(run_inverse(*p, nb, c + b0 * N, p->d_w, p->d_dth, c + b0 * N, cw.work, cw.lanes))))
                return r;
        }
        return DLT_OK;
    });
}

int leg2chebvals(int64_t N, int64_t batch, const double* c, double* v, hipStream_t stream) {
    int rc = check_size(N, batch);  // power-of-two sizes
    if (rc) return rc;
    if (batch == 0) return DLT_OK;
    if (!c || !v || overlap(c, v, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan(N, DLT_PREC_FP64, &p))) return rc;
    // Chebyshev coefficients (workspace), then the Taylor evaluation with all
    // offsets zero and one term pair: exactly the DCT-III onto the grid
    return run_call(6, *p, batch, c, v, stream, [&](CallWS& cw) -> int {
        int r = hip_status(run_fill_zero(cw.dth, N, cw.lanes.s));
        if (r) return r;
        for (int64_t b0 = 0; b0 < batch; b0 += cw.nb) {
            int64_t nb = std::min(cw.nb, batch - b0);
            double* chat = cw.work.chat;
            if ((r = hip_status(run_leg2cheb(*p, nb, c + b0 * N, N, chat, cw.work.schat, cw.work, cw.lanes)))) return r;
            if ((r = hip_status(run_ndct(*p, nb, chat, cw.work.schat, cw.dth, v + b0 * N, cw.work, cw.lanes, nullptr, 1))))
                return r;
        }
        return DLT_OK;
    });
}

int dlt_plan_query(int64_t N, int64_t* out, int max_fields) { return dlt_plan_query_ex(N, DLT_PREC_FP64, out, max_fields); }

static int plan_fields(const Plan* p, int64_t* out, int max_fields) {
    int64_t steps = 0, work = 0;
    for (int s = 0; s < p->near.nseg; ++s) {
        const int64_t rows = p->near.seg[s].jhi - p->near.seg[s].jlo;
        steps += rows * p->near.seg[s].nend;
        work += rows * std::max<int64_t>(0, p->near.seg[s].nend - p->nd);
    }
    const int64_t v[] = {p->L, p->nd, p->far.nterm, p->far.nblk, p->far.Mmax, p->near.nitems, p->near.jnear,
                         p->geo.N1, p->geo.N2, p->geo.colsA, p->geo.rowsB, p->tgB, p->tn_wg, p->tn_nrg, steps,
                         p->nodes.kb, (int64_t)p->ws_per_inst, work, p->tgA, (int64_t)WS_CAP,
                         (p->prec == PREC_FP64 && p->tol == 0) ? star_terms(5e-15) : 0};
    int n = (int)(sizeof(v) / sizeof(v[0]));
    for (int i = 0; i < n && i < max_fields; ++i) out[i] = v[i];
    return n;
}

int dlt_plan_query_ex(int64_t N, int prec, int64_t* out, int max_fields) {
    int rc = check_size(N, 1);
    if (rc) return rc;
    if ((rc = check_prec(prec))) return rc;
    if (!out || max_fields < 0) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan(N, prec, &p))) return rc;
    return plan_fields(p, out, max_fields);
}

int dlt_batch_grid(int64_t N, int inverse, int prec, int64_t* grid) {
    if (N < 1 || (inverse != 0 && inverse != 1) || !grid) return DLT_ERR_INVALID_ARG;
    if (N > DLT_MAX_N) return DLT_ERR_UNSUPPORTED;
    int rc;
    if ((rc = check_prec(prec))) return rc;
    const int64_t P = next_pow2(N);
    if (2 * P > DLT_MAX_N) {  // no larger candidate: never timed
        *grid = P;
        return DLT_OK;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DLT_ERR_HIP;
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.tuned.find(std::make_tuple(dev, inverse, P, prec));
    *grid = it == c.tuned.end() ? 0 : it->second;
    return DLT_OK;
}

int dlt_plan_query_tol(int64_t N, double eps, int64_t* out, int max_fields) {
    int rc = check_size(N, 1);
    if (rc) return rc;
    double tv;
    int ti;
    if ((rc = tol_step(eps, &tv, &ti))) return rc;
    if (!out || max_fields < 0) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan_tol(N, eps, &p))) return rc;
    return plan_fields(p, out, max_fields);
}

int dlt_trace_enable(int on) {
    trace_set(on != 0);
    return DLT_OK;
}

int dlt_trace_collect(int max_kernels, char* names, int name_len, double* total_ms, int64_t* counts) {
    if (max_kernels < 0 || name_len < 1 || (max_kernels > 0 && (!names || !total_ms || !counts)))
        return DLT_ERR_INVALID_ARG;
    std::vector<std::pair<std::string, std::pair<double, int64_t>>> v;
    if (trace_collect(v) != 0) return DLT_ERR_HIP;
    int n = 0;
    for (auto& kv : v) {
        if (n >= max_kernels) break;
        std::string s = kv.first.substr(0, (size_t)name_len - 1);
        memcpy(names + (size_t)n * name_len, s.c_str(), s.size() + 1);
        total_ms[n] = kv.second.first;
        counts[n] = kv.second.second;
        ++n;
    }
    return n;
}

int dlt_release(void) {
    Cache& c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    if (hipDeviceSynchronize() != hipSuccess) return DLT_ERR_HIP;
    for (auto& kv : c.plans) plan_free(*kv.second);
    c.plans.clear();
    for (auto& kv : c.ws)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    c.ws.clear();
    for (auto& kv : c.lanes) {
        for (int i = 0; i < LANE_SIDES; ++i)
            if (kv.second.side[i]) (void)hipStreamDestroy(kv.second.side[i]);
        for (int i = 0; i < LANE_EVENTS; ++i)
            if (kv.second.ev[i]) (void)hipEventDestroy(kv.second.ev[i]);
    }
    c.lanes.clear();
    c.graphs.clear();  // graph executables, their workspaces and descriptors
    for (auto& kv : c.calls)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    c.calls.clear();
    c.single.clear();
    c.tuned.clear();
    for (auto& kv : c.capture) (void)hipStreamDestroy(kv.second);
    c.capture.clear();
    return DLT_OK;
}

}  // extern "C"
