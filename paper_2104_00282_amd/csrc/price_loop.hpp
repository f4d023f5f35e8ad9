// Price-discovery loop (Algorithm 2, §5) as a state machine that requests one
// evaluation at a time, so that the same update logic drives one problem
// (ra_solve) and many problems evaluated together in one pass (ra_batch_solve).
//
// Every evaluation at prices p also carries the certificate of the point
// evaluated before it (the lower bound of its column-scaled allocation is
// formed in the same pass), so a point is certified one evaluation later.
//
// Price update: projected L-BFGS on f(p) = g(p)/n over p >= 0.  Direction
// d = -H grad f from the two-loop recursion with H0 = (s^T y / y^T y) I, with
// components that would push a zero price negative removed (memory cleared if
// d is then not a descent direction); trial p+ = max(p + lambda d, 0) with
// lambda = 1, or s0 |p|_inf / |d|_inf when the memory is empty (s0 = init_step,
// 0.1 when unset); Armijo test
// f(p+) <= f(p) + 1e-4 grad^T (p+ - p) with up to 20 halvings; a pair is kept
// if s^T y > 1e-12 |s| |y|.  When the line search fails, one projected
// subgradient step p+ = max(p - a_k q, 0), a_k = a0 / sqrt(k),
// a0 = 0.1 |p|_inf / |q|_inf, is taken instead (the fallback of §5); method 1
// uses only that step.  With stall_evals > 0 the loop also ends when the best
// certified relative gap has not improved by 0.1 % within that many passes
// (the column-scaling recovery has a floor, see ra_solve); with
// stall_restarts = k > 0 the first k such stalls instead restart the update
// from the best certified point with an empty memory (a new path to p*,
// with new chances of a tighter certificate), and a new window begins.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "resalloc.h"

namespace ra {

struct Point {
    std::vector<double> p;     // prices as evaluated (rounded to the problem dtype)
    std::vector<double> r;     // usage r(p)
    std::vector<double> grad;  // gradient of f = g / n, (R - r) / n
    double g = 0.0, f = 0.0;
    bool certified = false;
    double U = 0.0, gap = 0.0, rel = INFINITY;
};

class PriceLoop {
public:
    PriceLoop(int m, int64_t n, const double* R, const ra_solve_opts& o, const double* p0)
        : m_(m), n_(n), R_(R, R + m), o_(o), next_(p0, p0 + m), S_(o.lbfgs_mem, std::vector<double>(m)),
          Y_(o.lbfgs_mem, std::vector<double>(m)), rho_(o.lbfgs_mem), alpha_(o.lbfgs_mem), d_(m),
          step_(m), y_(m), q_(m)
    {
        for (double& v : next_) v = std::max(v, 0.0);
    }

    bool done() const { return state_ == DONE; }
    const std::vector<double>& next() const { return next_; }
    const Point* pending() const { return have_pend_ && !pend_.certified ? &pend_ : nullptr; }

    // Feed the evaluation of next(): prices as evaluated, g, r; and
    // sdu_prev = sum_i [u(t_i) - u(t~_i)] of pending() (ignored if none).
    void feed(const std::vector<double>& p_eval, double g, const double* r, double sdu_prev)
    {
        bool restart = false;
        if (have_pend_ && !pend_.certified) {
            certify(pend_, sdu_prev);
            last_cert_ = pend_;
            ++ncert_;
            if (!best_.certified || pend_.rel < best_.rel) {
                if (!best_.certified || pend_.rel < 0.999 * best_.rel) improved_at_ = evals_;
                best_ = pend_;
            }
            if (met(pend_)) {
                state_ = DONE;
                return;
            }
            if (o_.stall_evals > 0 && evals_ - improved_at_ >= o_.stall_evals) {
                if (restarts_ < o_.stall_restarts && (state_ == LINE_SEARCH ||
                                                      state_ == SUBGRADIENT)) {
                    ++restarts_;  // restart from the best point once e is taken in
                    restart = true;
                } else {
                    stalled_ = true;  // the best gap stopped improving: end here
                    state_ = DONE;
                    return;
                }
            }
        }
        // the evaluated point, built in a member so that its vectors keep
        // their storage from one pass to the next (no allocation per pass)
        Point& e = eval_;
        e.p.assign(p_eval.begin(), p_eval.end());
        e.g = g;
        e.f = g / (double)n_;
        e.r.assign(r, r + m_);
        e.grad.resize(m_);
        for (int j = 0; j < m_; ++j) e.grad[j] = (R_[j] - r[j]) / (double)n_;
        e.U = 0.0;
        e.gap = 0.0;
        e.rel = INFINITY;
        e.certified = false;
        ++evals_;
        const State was = state_;
        pend_ = e;
        have_pend_ = true;
        if (restart) {
            // a new window from the best certified point (the point just
            // evaluated is still certified by the next pass)
            improved_at_ = evals_;
            cur_ = best_;
            npairs_ = 0;
            start_iteration();
            return;
        }
        switch (was) {
        case INIT:
            cur_ = e;
            start_iteration();
            break;
        case LINE_SEARCH: {
            std::vector<double>& step = step_;
            for (int j = 0; j < m_; ++j) step[j] = e.p[j] - cur_.p[j];
            if (e.f <= cur_.f + 1e-4 * dot(cur_.grad, step)) {
                std::vector<double>& y = y_;
                for (int j = 0; j < m_; ++j) y[j] = e.grad[j] - cur_.grad[j];
                const double sy = dot(step, y);
                if (sy > 1e-12 * std::sqrt(dot(step, step) * dot(y, y))) {
                    const int M = (int)S_.size();
                    S_[head_] = step;
                    Y_[head_] = y;
                    rho_[head_] = 1.0 / sy;
                    head_ = (head_ + 1) % M;
                    npairs_ = std::min(npairs_ + 1, M);
                }
                cur_ = e;
                ++iters_;
                start_iteration();
            } else {
                lam_ *= 0.5;
                if (++ls_ >= 20) {
                    npairs_ = 0;
                    start_subgradient();
                } else {
                    next_line_search_point();
                }
            }
            break;
        }
        case SUBGRADIENT:
            cur_ = e;
            ++iters_;
            start_iteration();
            break;
        case FINAL:
        case DONE:
            state_ = DONE;
            break;
        }
    }

    // Outcome: the certified point with the smallest relative gap (or the
    // last point evaluated if none could be certified).
    const Point& result() const { return best_.certified ? best_ : pend_; }
    bool converged() const { return best_.certified && met(best_); }
    // Algorithm 2's stopping test on a certified point: relative gap, or the
    // absolute gap g - U(X~) when tol_abs is set
    bool met(const Point& e) const
    {
        return e.rel <= o_.tol_rel || (o_.tol_abs > 0.0 && e.gap <= o_.tol_abs);
    }
    int iters() const { return iters_; }
    int evals() const { return evals_; }
    int fallbacks() const { return fallbacks_; }
    int restarts() const { return restarts_; }
    bool stalled() const { return stalled_; }
    // The point certified by the last feed (valid when ncertified() grew).
    const Point& last_certified() const { return last_cert_; }
    int ncertified() const { return ncert_; }

    // Certificate from the pass's sum of utility lost by scaling:
    // gap = g - U(X~) = p^T (R - r) + sum_i [u(t_i) - u(t~_i)].
    void certify(Point& e, double sdu) const
    {
        double pq = 0.0;
        for (int j = 0; j < m_; ++j) pq += e.p[j] * (R_[j] - e.r[j]);
        e.gap = pq + sdu;
        e.U = e.g - e.gap;
        const double den = std::max(std::fabs(e.g), std::fabs(e.U));
        e.rel = e.gap / (den > 0 ? den : 1.0);
        e.certified = true;
    }

private:
    enum State { INIT, LINE_SEARCH, SUBGRADIENT, FINAL, DONE };

    static double dot(const std::vector<double>& a, const std::vector<double>& b)
    {
        double s = 0.0;
        for (size_t j = 0; j < a.size(); ++j) s += a[j] * b[j];
        return s;
    }
    static double inf_norm(const std::vector<double>& a)
    {
        double s = 0.0;
        for (double v : a) s = std::max(s, std::fabs(v));
        return s;
    }
    bool budget_left() const { return o_.max_evals == 0 || evals_ < o_.max_evals; }

    void go_final()
    {
        if (have_pend_ && !pend_.certified && budget_left()) {
            next_ = pend_.p;
            state_ = FINAL;
        } else {
            state_ = DONE;
        }
    }

    void start_iteration()
    {
        if (iters_ >= o_.max_iter || !budget_left()) {
            go_final();
            return;
        }
        if (o_.method == 1) {
            start_subgradient();
            return;
        }
        const int M = (int)S_.size();
        std::vector<double>& q = q_;
        q = cur_.grad;
        for (int h = 0; h < npairs_; ++h) {
            const int s = (head_ - 1 - h + M) % M;
            alpha_[h] = rho_[s] * dot(S_[s], q);
            for (int j = 0; j < m_; ++j) q[j] -= alpha_[h] * Y_[s][j];
        }
        if (npairs_ > 0) {
            const int s = (head_ - 1 + M) % M;
            const double gam = dot(S_[s], Y_[s]) / dot(Y_[s], Y_[s]);
            for (int j = 0; j < m_; ++j) q[j] *= gam;
        }
        for (int h = npairs_ - 1; h >= 0; --h) {
            const int s = (head_ - 1 - h + M) % M;
            const double b = rho_[s] * dot(Y_[s], q);
            for (int j = 0; j < m_; ++j) q[j] += S_[s][j] * (alpha_[h] - b);
        }
        for (int j = 0; j < m_; ++j) d_[j] = (cur_.p[j] <= 0.0 && q[j] > 0.0) ? 0.0 : -q[j];
        if (dot(d_, cur_.grad) >= 0.0) {
            npairs_ = 0;
            for (int j = 0; j < m_; ++j)
                d_[j] = (cur_.p[j] <= 0.0 && cur_.grad[j] > 0.0) ? 0.0 : -cur_.grad[j];
        }
        const double dn = inf_norm(d_);
        if (dn == 0.0) {
            go_final();
            return;
        }
        lam_ = 1.0;
        if (npairs_ == 0) {
            const double pi = inf_norm(cur_.p);
            const double s0 = o_.init_step > 0.0 ? o_.init_step : 0.1;
            lam_ = s0 * (pi > 0.0 ? pi : 1.0) / dn;
        }
        ls_ = 0;
        state_ = LINE_SEARCH;
        next_line_search_point();
    }

    void next_line_search_point()
    {
        if (!budget_left()) {
            go_final();
            return;
        }
        for (int j = 0; j < m_; ++j) next_[j] = std::max(cur_.p[j] + lam_ * d_[j], 0.0);
    }

    void start_subgradient()
    {
        if (!budget_left()) {
            go_final();
            return;
        }
        ++sg_steps_;
        ++fallbacks_;
        const double gi = inf_norm(cur_.grad), pi = inf_norm(cur_.p);
        const double a0 = gi > 0.0 ? 0.1 * (pi > 0.0 ? pi : 1.0) / gi : 0.0;
        const double ak = a0 / std::sqrt((double)sg_steps_);
        for (int j = 0; j < m_; ++j) next_[j] = std::max(cur_.p[j] - ak * cur_.grad[j], 0.0);
        state_ = SUBGRADIENT;
    }

    int m_;
    int64_t n_;
    std::vector<double> R_;
    ra_solve_opts o_;
    State state_ = INIT;
    std::vector<double> next_;
    Point cur_, pend_, best_, last_cert_;
    int ncert_ = 0;
    bool have_pend_ = false;
    std::vector<std::vector<double>> S_, Y_;
    std::vector<double> rho_, alpha_, d_;
    // scratch reused by every pass: the evaluated point, the step and
    // gradient change of a line-search trial, the two-loop vector
    Point eval_;
    std::vector<double> step_, y_, q_;
    int npairs_ = 0, head_ = 0, ls_ = 0;
    double lam_ = 1.0;
    int evals_ = 0, iters_ = 0, fallbacks_ = 0, sg_steps_ = 0, restarts_ = 0;
    int improved_at_ = 0;
    bool stalled_ = false;
};

}  // namespace ra
