// C ABI: argument validation, plan and workspace caches, and the order in
// which the pipelines are enqueued.  Declared in include/dlt.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <utility>

#include "../../include/dlt.h"
#include "dlt_kernels.hpp"

using namespace dlt;

namespace {

struct Cache {
    std::mutex mu;
    std::map<std::tuple<int, int64_t, int>, std::unique_ptr<Plan>> plans;  // (device, N, precision)
    struct WS {
        void* ptr = nullptr;
        size_t bytes = 0;
    };
    std::map<std::pair<int, hipStream_t>, WS> ws;  // (device, stream)
    std::map<std::pair<int, hipStream_t>, Lanes> lanes;  // (device, stream): side streams, events
};

Cache& cache() {
    static Cache* c = new Cache();  // never destroyed: device memory goes with the process
    return *c;
}

const size_t WS_CAP = size_t(6) << 30;  // per-stream workspace bound; larger batches run in slices

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

int check_prec(int prec) {
    return (prec == DLT_PREC_FP64 || prec == DLT_PREC_FP32_BULK || prec == DLT_PREC_FP64_RELAXED) ? DLT_OK
                                                                                                : DLT_ERR_INVALID_ARG;
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
    double* nscr;  // node scratch
    int64_t nb;  // instances per slice
    Lanes lanes;
};

int setup_call(const Plan& p, int64_t batch, hipStream_t s, CallWS& cw) {
    size_t per = p.ws_per_inst;
    int64_t nb = batch;
    if (per > 0 && (size_t)nb * per > WS_CAP) nb = (int64_t)(WS_CAP / per);
    if (batch > 0 && nb < 1) nb = 1;
    size_t shared = p.ws_shared + (size_t)64 * NODE_PARTS_MAX * 8 * sizeof(double);
    void* base = nullptr;
    int rc = get_ws(s, shared + work_bytes(p, nb), &base);
    if (rc) return rc;
    size_t vecb = ((size_t)p.N * sizeof(double) + 255) & ~size_t(255);
    cw.theta = (double*)base;
    cw.w = (double*)((char*)base + vecb);
    cw.dth = (double*)((char*)base + 2 * vecb);
    cw.nscr = (double*)((char*)base + 3 * vecb);
    work_carve(p, nb, (char*)base + shared, cw.work);
    cw.nb = nb;
    return get_lanes(s, &cw.lanes);
}

int hip_status(hipError_t e) { return e == hipSuccess ? DLT_OK : DLT_ERR_HIP; }

}  // namespace

extern "C" {

const char* dlt_status_string(int st) {
    switch (st) {
        case DLT_OK: return "ok";
        case DLT_ERR_INVALID_ARG: return "invalid argument";
        case DLT_ERR_UNSUPPORTED: return "unsupported size";
        case DLT_ERR_HIP: return "HIP runtime error";
        case DLT_ERR_NOMEM: return "out of device memory";
        default: return "unknown status";
    }
}

int leg_nodes_weights(int64_t N, int64_t batch, double* theta, double* w, double* dtheta, hipStream_t stream) {
    int rc = check_size(N, batch);
    if (rc) return rc;
    if (batch == 0 || (!theta && !w && !dtheta)) return DLT_OK;
    size_t bytes = (size_t)N * sizeof(double) * (size_t)batch;
    if ((theta && w && overlap(theta, w, bytes)) || (theta && dtheta && overlap(theta, dtheta, bytes)) ||
        (w && dtheta && overlap(w, dtheta, bytes)))
        return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan(N, DLT_PREC_FP64, &p))) return rc;
    CallWS cw;
    if ((rc = setup_call(*p, 0, stream, cw))) return rc;
    if ((rc = hip_status(run_nodes(*p, theta, w, dtheta, cw.nscr, cw.lanes)))) return rc;
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

int leg2cheb_ex(int64_t N, int64_t batch, const double* c, double* chat, int prec, hipStream_t stream) {
    int rc = check_size(N, batch);
    if (rc) return rc;
    if ((rc = check_prec(prec))) return rc;
    if (batch == 0) return DLT_OK;
    if (!c || !chat || overlap(c, chat, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan(N, prec, &p))) return rc;
    CallWS cw;
    if ((rc = setup_call(*p, batch, stream, cw))) return rc;
    for (int64_t b0 = 0; b0 < batch; b0 += cw.nb) {
        int64_t nb = std::min(cw.nb, batch - b0);
        if ((rc = hip_status(run_leg2cheb(*p, nb, c + b0 * N, N, chat + b0 * N, N, cw.work, cw.lanes)))) return rc;
    }
    return DLT_OK;
}

int cheb_eval_leggrid(int64_t N, int64_t batch, const double* chat, double* f, hipStream_t stream) {
    return cheb_eval_leggrid_ex(N, batch, chat, f, DLT_PREC_FP64, stream);
}

int cheb_eval_leggrid_ex(int64_t N, int64_t batch, const double* chat, double* f, int prec, hipStream_t stream) {
    int rc = check_size(N, batch);
    if (rc) return rc;
    if ((rc = check_prec(prec))) return rc;
    if (batch == 0) return DLT_OK;
    if (!chat || !f || overlap(chat, f, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan(N, prec, &p))) return rc;
    CallWS cw;
    if ((rc = setup_call(*p, batch, stream, cw))) return rc;
    if ((rc = hip_status(run_nodes(*p, nullptr, nullptr, cw.dth, cw.nscr, cw.lanes)))) return rc;
    for (int64_t b0 = 0; b0 < batch; b0 += cw.nb) {
        int64_t nb = std::min(cw.nb, batch - b0);
        if ((rc = hip_status(run_ndct(*p, nb, chat + b0 * N, N, cw.dth, f + b0 * N, cw.work, cw.lanes)))) return rc;
    }
    return DLT_OK;
}

int dlt_forward(int64_t N, int64_t batch, const double* c, double* f, hipStream_t stream) {
    return dlt_forward_ex(N, batch, c, f, DLT_PREC_FP64, stream);
}

int dlt_forward_ex(int64_t N, int64_t batch, const double* c, double* f, int prec, hipStream_t stream) {
    int rc = check_size(N, batch);
    if (rc) return rc;
    if ((rc = check_prec(prec))) return rc;
    if (batch == 0) return DLT_OK;
    if (!c || !f || overlap(c, f, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan(N, prec, &p))) return rc;
    CallWS cw;
    if ((rc = setup_call(*p, batch, stream, cw))) return rc;
    // the nodes are needed only by the Taylor evaluation: they run on the
    // first side stream beside the conversion of the first slice
    const Lanes& L = cw.lanes;
    const hipStream_t sn = L.aux(0);
    if (hipEventRecord(L.ev[10], stream) != hipSuccess || hipStreamWaitEvent(sn, L.ev[10], 0) != hipSuccess)
        return DLT_ERR_HIP;
    if ((rc = hip_status(run_nodes(*p, nullptr, nullptr, cw.dth, cw.nscr, L.on(sn))))) return rc;
    if (hipEventRecord(L.ev[11], sn) != hipSuccess) return DLT_ERR_HIP;
    for (int64_t b0 = 0; b0 < batch; b0 += cw.nb) {
        int64_t nb = std::min(cw.nb, batch - b0);
        // Chebyshev coefficients of the slice, stride N, in the workspace
        double* chat = cw.work.chat;
        if ((rc = hip_status(run_leg2cheb(*p, nb, c + b0 * N, N, chat, cw.work.schat, cw.work, L)))) return rc;
        if (b0 == 0 && hipStreamWaitEvent(stream, L.ev[11], 0) != hipSuccess) return DLT_ERR_HIP;
        if ((rc = hip_status(run_ndct(*p, nb, chat, cw.work.schat, cw.dth, f + b0 * N, cw.work, L)))) return rc;
    }
    return DLT_OK;
}

int dlt_inverse(int64_t N, int64_t batch, const double* f, double* c, hipStream_t stream) {
    return dlt_inverse_ex(N, batch, f, c, DLT_PREC_FP64, stream);
}

int dlt_inverse_ex(int64_t N, int64_t batch, const double* f, double* c, int prec, hipStream_t stream) {
    int rc = check_size(N, batch);
    if (rc) return rc;
    if ((rc = check_prec(prec))) return rc;
    if (batch == 0) return DLT_OK;
    if (!f || !c || overlap(f, c, (size_t)N * batch * sizeof(double))) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan(N, prec, &p))) return rc;
    CallWS cw;
    if ((rc = setup_call(*p, batch, stream, cw))) return rc;
    if ((rc = hip_status(run_nodes(*p, nullptr, cw.w, cw.dth, cw.nscr, cw.lanes)))) return rc;
    for (int64_t b0 = 0; b0 < batch; b0 += cw.nb) {
        int64_t nb = std::min(cw.nb, batch - b0);
        if ((rc = hip_status(run_inverse(*p, nb, f + b0 * N, cw.w, cw.dth, c + b0 * N, cw.work, cw.lanes)))) return rc;
    }
    return DLT_OK;
}

int dlt_plan_query(int64_t N, int64_t* out, int max_fields) { return dlt_plan_query_ex(N, DLT_PREC_FP64, out, max_fields); }

int dlt_plan_query_ex(int64_t N, int prec, int64_t* out, int max_fields) {
    int rc = check_size(N, 1);
    if (rc) return rc;
    if ((rc = check_prec(prec))) return rc;
    if (!out || max_fields < 0) return DLT_ERR_INVALID_ARG;
    Plan* p;
    if ((rc = get_plan(N, prec, &p))) return rc;
    int64_t steps = 0, work = 0;
    for (int s = 0; s < p->near.nseg; ++s) {
        const int64_t rows = p->near.seg[s].jhi - p->near.seg[s].jlo;
        steps += rows * p->near.seg[s].nend;
        work += rows * std::max<int64_t>(0, p->near.seg[s].nend - p->nd);
    }
    const int64_t v[] = {p->L, p->nd, p->far.nterm, p->far.nblk, p->far.Mmax, p->near.nitems, p->near.jnear,
                         p->geo.N1, p->geo.N2, p->geo.colsA, p->geo.rowsB, p->tgB, p->tn_wg, p->tn_nrg, steps,
                         p->nodes.kb, (int64_t)p->ws_per_inst, work, p->tgA};
    int n = (int)(sizeof(v) / sizeof(v[0]));
    for (int i = 0; i < n && i < max_fields; ++i) out[i] = v[i];
    return n;
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
    return DLT_OK;
}

}  // extern "C"
