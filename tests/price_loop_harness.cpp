// CPU harness for the host price loop (paper_2104_00282_amd/csrc/price_loop.hpp):
// drives it with fake evaluators and prints one line of results.
//   f(p) = g/n = 0.5 (p - c)^T D (p - c) + f0, so grad f = D (p - c) and
//   r = R - n grad f; the certificate's loss term is k |p - pstar|^2 with
//   pstar = max(c, 0) (the projected minimiser), so the gap vanishes there.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "price_loop.hpp"

int main(int argc, char** argv)
{
    const char* mode = argc > 1 ? argv[1] : "interior";
    const int m = 5;
    const int64_t n = 1000;
    std::vector<double> R(m, 100.0), c(m), D(m);
    for (int j = 0; j < m; ++j) {
        c[j] = 1.0 + 0.5 * j;
        D[j] = 1.0 + j;
    }
    if (!std::strcmp(mode, "boundary")) c[2] = -0.7;  // minimiser outside p >= 0
    ra_solve_opts o;
    o.tol_rel = 1e-10;
    o.max_iter = 200;
    o.lbfgs_mem = 10;
    o.method = !std::strcmp(mode, "subgradient") ? 1 : 0;
    o.init = 0;
    o.use_graph = 0;
    o.verbose = 0;
    o.max_evals = !std::strcmp(mode, "budget") ? 7 : 0;
    const bool stall = !std::strcmp(mode, "stall") || !std::strcmp(mode, "stall_restart");
    o.stall_evals = stall ? 25 : 0;
    o.stall_restarts = !std::strcmp(mode, "stall_restart") ? 3 : 0;
    o.init_step = 0.0;
    o.tol_abs = 0.0;
    if (!std::strcmp(mode, "subgradient")) o.max_iter = 400;
    std::vector<double> p0(m, 3.0);
    ra::PriceLoop L(m, n, R.data(), o, p0.data());
    const double f0 = 2.0;
    int calls = 0;
    bool restart_ok = true;
    int restart_checks = 0;
    while (!L.done() && calls < 100000) {
        const std::vector<double>& p = L.next();
        std::vector<double> r(m);
        double f = f0, dist = 0.0;
        for (int j = 0; j < m; ++j) {
            const double e = p[j] - c[j];
            f += 0.5 * D[j] * e * e;
            double gj = D[j] * e;
            // inconsistent gradient: wrong sign on one coordinate
            if (!std::strcmp(mode, "badgrad") && j == 0) gj = -gj;
            // stall: a small wobble keeps the loop moving around the minimiser
            if (stall) gj += 1e-3 * std::sin(7.0 * calls + j);
            r[j] = R[j] - (double)n * gj;
            const double ps = std::max(c[j], 0.0);
            dist += (p[j] - ps) * (p[j] - ps);
        }
        // stall: the certificate never gets better than a floor
        double sdu = 0.0;
        const ra::Point* prev = L.pending();
        if (prev) {
            double dprev = 0.0, pq = 0.0;
            for (int j = 0; j < m; ++j) {
                const double ps = std::max(c[j], 0.0);
                dprev += (prev->p[j] - ps) * (prev->p[j] - ps);
                pq += prev->p[j] * (R[j] - prev->r[j]);
            }
            // gap(prev) = 50 n |prev - pstar|^2 (+ a floor in stall mode)
            double want = 50.0 * (double)n * dprev;
            if (stall) want += 1.0;
            sdu = want - pq;
        }
        const int rs0 = L.restarts();
        L.feed(p, f * (double)n, r.data(), sdu);
        ++calls;
        if (L.restarts() > rs0 && !L.done()) {
            // a restart: the next point is the projected steepest-descent
            // step from the best certified point with the empty-memory length
            const ra::Point& b = L.result();
            double pi = 0.0, gi = 0.0;
            for (int j = 0; j < m; ++j) {
                pi = std::max(pi, std::fabs(b.p[j]));
                gi = std::max(gi, std::fabs(b.grad[j]));
            }
            const double lam = 0.1 * pi / gi;
            bool ok = b.certified;
            for (int j = 0; j < m; ++j) {
                const double want = std::max(b.p[j] - lam * b.grad[j], 0.0);
                ok = ok && std::fabs(L.next()[j] - want) <= 1e-12 * (1.0 + std::fabs(want));
            }
            restart_ok = restart_ok && ok;
            ++restart_checks;
        }
        (void)dist;
    }
    const ra::Point& res = L.result();
    double err = 0.0;
    for (int j = 0; j < m; ++j) err = std::max(err, std::fabs(res.p[j] - std::max(c[j], 0.0)));
    std::printf("done=%d converged=%d stalled=%d iters=%d evals=%d fallbacks=%d calls=%d "
                "rel=%.3e err=%.3e restarts=%d restart_checks=%d restart_ok=%d\n",
                (int)L.done(), (int)L.converged(), (int)L.stalled(), L.iters(), L.evals(),
                L.fallbacks(), calls, res.rel, err, L.restarts(), restart_checks,
                (int)restart_ok);
    return 0;
}
