// Internal definitions shared by the host sources of libresalloc.so.
// Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "dev_loop.hpp"
#include "host_pool.hpp"
#include "ra_kernels.h"
#include "resalloc.h"

struct ra_ctx {
    int dev = 0;
    int cus = 1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int live_problems = 0;  // problems created on this context and not destroyed
    bool closed = false;    // ra_destroy called; freed when the last problem goes
    double* scratch = nullptr; // device address of this device's static scratch
    bool timing = false;    // bracket dual-kernel launches with events
    bool timed_pending = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
    // batched solver: tuned launch shapes by batch signature, a shape fixed
    // by the caller (ra_batch_set_shape), and the record of the last tuning
    std::map<std::string, ra::BatchTuned> batch_tuned;
    bool batch_fixed = false;
    ra::BatchTuned batch_fixed_shape;
    std::string batch_tune_log;
    std::shared_ptr<void> batch_ws;  // the batched solver's workspace, reused by later batches
    std::shared_ptr<void> batch_ws2;  // the second group's workspace (batches of 16 or more)
    std::unique_ptr<ra::HostPool> pool;      // host threads of the batched solver
    void* feat_ws = nullptr;  // warm-start features: sampled keys and block partials
};

struct ra_problem {
    ra_ctx* ctx = nullptr;
    int64_t n = 0;
    int m = 0;
    int dt = 0;  // 0 = FP32, 1 = FP64
    const void* T = nullptr;
    bool vec_ok = false;
    void* prm = nullptr;
    std::vector<double> R;
    double* Rdev = nullptr;
    double eps = 0.0;
    int grid = 1;
    int lgrid = 1;
    double* partial = nullptr;
    double* partial2 = nullptr;
    double* dout = nullptr;     // r[0..m), sum v, sum u(t~), sum u(t) - u(t~)
    void* pblock = nullptr;
    void* h_pblock = nullptr;
    double* h_out = nullptr;    // fine-grained host memory: m + 3 results, then the flag
    unsigned* h_flag = nullptr; // set to 1 by the reduction when a solver pass is done
    unsigned* ticket = nullptr; // device block counter of that reduction
    bool alpha_fair = false;    // some job has an alpha-fair utility other than log
    void* dem = nullptr;        // per-job demands (dtype, n), or NULL
    const void* dvec = nullptr; // per-job demand vectors (dtype, n x m, borrowed), or NULL
    int grid_cap = 1;           // block rows `partial` holds
    void* w0 = nullptr;         // the weights as packed before demands were applied
    int16_t* jpair_ws = nullptr;
    void* tpair_ws = nullptr;
    void* xpair_ws = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    // device price loop: its state, the prices it writes for the next pass,
    // pinned status words, and the captured graph of a chunk of passes
    ra::DevLoop* dloop = nullptr;
    void* dprices = nullptr;
    ra::DevStatus* h_dl = nullptr;
    void* h_dlstage = nullptr;  // pinned: the header and first prices of a solve
    hipGraphExec_t dl_gexec = nullptr;
    hipGraph_t dl_graph = nullptr;
};

namespace ra {

// Record a failure on ctx (printf-style detail) and return st.
inline ra_status fail(ra_ctx* ctx, ra_status st, const char* fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

#define RA_HIP(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::ra::fail((ctx), e_ == hipErrorOutOfMemory ? RA_ENOMEM : RA_EDEVICE, "%s: %s", \
                        #call, hipGetErrorString(e_));                                      \
    } while (0)

// Spin until a kernel has set the pinned completion flag to 1 (runtime.hip);
// a stream that ends or fails without it gives RA_EDEVICE.
ra_status wait_flag(ra_ctx* ctx, unsigned* flag);

// Learned warm start (mlp.hip)
ra_status features_into(ra_problem* P, float* feat);
ra_status predict_prices(ra_mlp* N, ra_problem* P, std::vector<double>& p0);
int mlp_out_dim(const ra_mlp* N);
int mlp_in_dim(const ra_mlp* N);

}  // namespace ra
