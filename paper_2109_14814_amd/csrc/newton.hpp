// newton.hpp -- the damped Newton iteration of Sec. 7 shared by the
// refinement of linear patches (refine.hip) and of Fourier-Taylor charts
// (fourier_taylor.hip): x <- x - alpha Df^{-1} f with alpha reset to alpha0
// after every accepted point and halved after every trial point whose
// r = |f|^2 is not below the current one.
#pragma once

#include "ms_internal.hpp"

namespace ms {

enum { NW_RUNNING = -1, NW_CONVERGED = 0, NW_LIMIT = 1, NW_STALLED = 2, NW_SINGULAR = 3, NW_NONFINITE = 4 };

struct NewtonState {
    double *p, *q, *delta, *fp;   // K x 4
    double *rp, *alpha;           // K
    int32_t *status, *trials, *based;
};

struct NewtonCfg {
    double tol2, alpha0, alpha_min;
    int32_t max_trials;
};

// Solve M z = r (4 x 4) by Gaussian elimination with partial pivoting: pivot
// = first row of largest magnitude; an exact zero pivot means singular.
MS_D bool gepp4(double M[4][4], double r[4], double z[4])
{
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int piv = k;
        double best = fabs(M[k][k]);
#pragma unroll
        for (int i = k + 1; i < 4; ++i) {
            double v = fabs(M[i][k]);
            if (v > best) { best = v; piv = i; }
        }
#pragma unroll
        for (int i = k + 1; i < 4; ++i) {
            bool sw = piv == i;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                double x = M[k][j], y = M[i][j];
                M[k][j] = sw ? y : x;
                M[i][j] = sw ? x : y;
            }
            double x = r[k], y = r[i];
            r[k] = sw ? y : x;
            r[i] = sw ? x : y;
        }
        ok = ok && (M[k][k] != 0.0);
#pragma unroll
        for (int i = k + 1; i < 4; ++i) {
            double l = M[i][k] / M[k][k];
#pragma unroll
            for (int j = k + 1; j < 4; ++j) M[i][j] = M[i][j] - l * M[k][j];
            r[i] = r[i] - l * r[k];
        }
    }
#pragma unroll
    for (int k = 3; k >= 0; --k) {
        double acc = 0.0;
#pragma unroll
        for (int j = k + 1; j < 4; ++j) acc = acc + M[k][j] * z[j];
        z[k] = (r[k] - acc) / M[k][k];
    }
    return ok;
}


// One decision for problem k, given f and Df = M at its trial point q:
// accept or reject q, then either stop (status >= 0) or set the next trial
// point q = p + alpha delta.
MS_D void newton_decide(int64_t k, const double f[4], double M[4][4], const NewtonState &ns, const NewtonCfg &cfg)
{
    double r = 0.0;
    for (int c = 0; c < 4; ++c) r += f[c] * f[c];
    int st = NW_RUNNING;
    bool accept;
    if (!ns.based[k]) {
        accept = true;
        if (!isfinite(r)) st = NW_NONFINITE;
    } else {
        ns.trials[k] += 1;
        accept = r < ns.rp[k];
    }
    if (accept && st == NW_RUNNING) {
        for (int c = 0; c < 4; ++c) {
            ns.p[4 * k + c] = ns.q[4 * k + c];
            ns.fp[4 * k + c] = f[c];
        }
        ns.rp[k] = r;
        ns.alpha[k] = cfg.alpha0;
        ns.based[k] = 1;
        if (r <= cfg.tol2) {
            st = NW_CONVERGED;
        } else {
            double rhs[4], z[4];
            for (int c = 0; c < 4; ++c) rhs[c] = -f[c];
            if (!gepp4(M, rhs, z)) st = NW_SINGULAR;
            else
                for (int c = 0; c < 4; ++c) ns.delta[4 * k + c] = z[c];
        }
    } else if (st == NW_RUNNING) {
        double al = ns.alpha[k] * 0.5;
        ns.alpha[k] = al;
        if (al < cfg.alpha_min) st = NW_STALLED;
    }
    if (st == NW_RUNNING && ns.trials[k] >= cfg.max_trials) st = NW_LIMIT;
    if (st == NW_RUNNING) {
        double al = ns.alpha[k];
        for (int c = 0; c < 4; ++c) ns.q[4 * k + c] = ns.p[4 * k + c] + al * ns.delta[4 * k + c];
    }
    ns.status[k] = st;
}

MS_D void newton_init(int64_t k, const double *x0, const NewtonState &ns)
{
    for (int c = 0; c < 4; ++c) ns.q[4 * k + c] = x0[4 * k + c];
    ns.status[k] = NW_RUNNING;
    ns.trials[k] = 0;
    ns.based[k] = 0;
}

// Final point (the last accepted one, else the start), f, r, status, trials.
MS_D void newton_finish(int64_t k, const NewtonState &ns, double *x_out, double *f_out, double *r_out,
                        int32_t *st_out, int32_t *tr_out)
{
    int st = ns.status[k] < 0 ? NW_LIMIT : ns.status[k];
    const bool based = ns.based[k] != 0;
    for (int c = 0; c < 4; ++c) {
        x_out[4 * k + c] = based ? ns.p[4 * k + c] : ns.q[4 * k + c];
        if (f_out) f_out[4 * k + c] = based ? ns.fp[4 * k + c] : NAN;
    }
    if (r_out) r_out[k] = based ? ns.rp[k] : NAN;
    if (st_out) st_out[k] = st;
    if (tr_out) tr_out[k] = ns.trials[k];
}

}  // namespace ms
