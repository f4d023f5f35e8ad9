// State of the price-discovery loop when it runs on the device (one wave of
// the reduction kernel that follows each dual pass takes the step), so that a
// solve is a replayed graph of passes with no host round trip between them.  The update is the host PriceLoop's (price_loop.hpp): projected
// L-BFGS on g/n with Armijo backtracking, the projected subgradient fallback,
// one-pass-late certificates, stall stops and restarts, budget stops.  Lane j of the wave
// holds coordinate j (m <= 64, the vectorised kernels' classes).
#pragma once

#include <cstdint>

namespace ra {

constexpr int DL_MAX_M = 64;    // coordinates (one per lane)
constexpr int DL_MAX_MEM = 32;  // L-BFGS pairs

struct DevPoint {
    double p[DL_MAX_M];     // prices as evaluated (rounded to FP32)
    double r[DL_MAX_M];     // usage r(p)
    double grad[DL_MAX_M];  // (R - r) / n
    double g, f, U, gap, rel;
    int certified;
    int pad;
};

// Everything the host writes before a solve comes first (the header), so
// that it is one small copy; the rest is initialised by the kernel as the
// loop reaches it.
struct DevLoop {
    // ---- header: written by the host before the first pass
    int m, mem, method, max_iter, max_evals, stall_evals, stall_restarts;
    double n, tol_rel, tol_abs, init_step;
    double R[DL_MAX_M];
    double pe[DL_MAX_M];  // prices of the pass in flight, as rounded for it
    double pR;            // p^T R of those prices
    int state;            // 0 INIT, 1 LINE_SEARCH, 2 SUBGRADIENT, 3 FINAL, 4 DONE
    int done;             // set when the loop has ended: later kernels return at once
    int error;            // 1: non-finite dual value, usage or gap
    int have_pend, npairs, head, ls, evals, iters, fallbacks, sg_steps, improved_at, ncert,
        stalled, converged, restarts;
    double lam;
    // ---- result: written by the step that ends the loop
    double res_p[DL_MAX_M];
    double res_g, res_U, res_rel;
    int res_certified;
    int pad;
    // ---- working state
    DevPoint cur, pend, best;
    double next[DL_MAX_M];
    double d[DL_MAX_M];
    double S[DL_MAX_MEM][DL_MAX_M], Y[DL_MAX_MEM][DL_MAX_M];
    double rho[DL_MAX_MEM], alpha[DL_MAX_MEM];
    // ---- not staged: blocks of the reduction that have finished (zero
    // between launches; the last block resets it)
    unsigned ticket;
    unsigned pad2;
};

// What the host waits on, in pinned host memory: the number of passes taken
// so far, and when the loop has ended, its outcome, published last by done.
struct DevStatus {
    int done;  // 0 running, 1 ended, 2 ended on a non-finite value
    int passes;
    int iters, evals, fallbacks, converged, certified, pad;
    double g, U, rel;
    double p[DL_MAX_M];
};

}  // namespace ra
