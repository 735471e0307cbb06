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
    int64_t sX, sv, sitems, snear, sdense, schat, svec, spart;  // per-instance strides (elements)
};
size_t work_bytes(const Plan& p, int64_t nb);
void work_carve(const Plan& p, int64_t nb, void* base, Work& w);

// theta, w, dtheta (any may be null) for the plan's N
// `scratch` holds kb * NODE_PARTS_MAX * 8 doubles
constexpr int NODE_PARTS_MAX = 64;
hipError_t run_nodes(const Plan& p, double* theta, double* w, double* dth, double* scratch, hipStream_t s);
// Input-independent plan data formed on the device once per plan (and its
// sub-plans): the near-field states at every chunk start.  Synchronous.
hipError_t plan_prepare(Plan& p);
// chat = M c for nb instances (batch strides cs, hs in elements)
hipError_t run_leg2cheb(const Plan& p, int64_t nb, const double* c, int64_t cs, double* chat, int64_t hs, Work& w,
                        hipStream_t s);
// out = M^T y (times n + 1/2 when half != 0)
hipError_t run_leg2cheb_t(const Plan& p, int64_t nb, const double* y, int64_t ys, double* out, int64_t os, int half,
                          Work& w, hipStream_t s);
// f = sum_n chat_n cos(n theta^leg), dth = theta^leg - theta^cheb1
hipError_t run_ndct(const Plan& p, int64_t nb, const double* chat, int64_t hs, const double* dth, double* f,
                    Work& w, hipStream_t s);

// c = D_s M^T T^T D_w f (inverse transform), wts/dth from the nodes
hipError_t run_inverse(const Plan& p, int64_t nb, const double* f, const double* wts, const double* dth,
                       double* c, Work& w, hipStream_t s);

// kernel trace (events around every launch while enabled)
bool trace_on();
void trace_set(bool enable);
int trace_collect(std::vector<std::pair<std::string, std::pair<double, int64_t>>>& out);

}  // namespace dlt
