// refine.hip -- the refinement problem of Sec. 7 on the GPU.
//
// For two parameterised patches x_u(th1, s1) = bu + th1 du1 + s1 du2 and
// x_s(th2, s2) = bs + th2 ds1 + s2 ds2, the mismatch is
//   f(th1, s1, th2, s2) = F^{n_u}(x_u(th1, s1)) - F^{n_s}(x_s(th2, s2)),
// with F the stroboscopic map integrated by the fixed-step order-8 method.
//   * residual: f and r = |f|^2;
//   * tangent: the Jacobian J = df/d(th1, s1, th2, s2, e) by integrating the
//     variational equations with the same method (the state transition
//     matrices DF^m of Sec. 7, applied to the patch directions), exactly the
//     derivative of the discrete map; e enters through w(f) = 1/(1 + e cos f);
//   * adjoint: the gradient of r by the discrete adjoint (transpose) of every
//     Runge-Kutta step, run backwards from the seed dr/dF = +-2f, with the
//     forward states kept only every `ckpt_every` steps and recomputed one
//     window of segments at a time;
//   * damped Newton (Sec. 7): x <- x - alpha Df^{-1} f, alpha halved until r
//     decreases.
//
// One thread per trajectory (hit, side) for the state pass, per (trajectory,
// tangent column) for the tangent pass and per (step, trajectory, column) for
// the adjoint's step Jacobians; blocks of one wave, so that the few hundred to
// few thousand trajectories spread over the compute units.
#include <math.h>
#include <string.h>

#include "newton.hpp"
#include "rk8_core.hpp"

namespace ms {

// The tableau in constant memory, initialised at compile time (every device
// holds it from the moment the code object is loaded).
__constant__ Tableau c_cv = cv_make_tableau();

namespace {

constexpr int S = RK_S;
constexpr int RF_BLOCK = 64;

struct SideMap {
    const double *w;       // stage values w(f), steps x S (in the workspace)
    const double *dwde;    // stage values dw/de, steps x S (in the workspace)
    double h;              // signed step
    int64_t nsteps;
    int32_t steps;         // steps per period
    int32_t pad;
};

struct RefArgs {
    const double *params;   // K x 4 (th1, s1, th2, s2)
    const double *U, *Sp;   // patches, 12 doubles each (base, d1, d2)
    int64_t K;
    int64_t pstride;        // doubles between consecutive hits' patches (0 or 12)
    Model md;
    SideMap side[2];        // 0: unstable side (x_u), 1: stable side (x_s)
    int64_t ck;             // checkpoint interval (steps)
    double *ckpt;           // n_ck x 2K x 4 (adjoint; NULL otherwise)
    double *yend;           // 2K x 4
    double *dend;           // 3 x 2K x 4 (tangent)
    double *gpart;          // 2K x 3 (adjoint)
    const int32_t *status;  // K Newton status words; only hits with status < 0 run (NULL: all run)
};

MS_D void store_d4(double *p, const double y[4])
{
    double2 *o = reinterpret_cast<double2 *>(p);
    o[0] = make_double2(y[0], y[1]);
    o[1] = make_double2(y[2], y[3]);
}

// Start of trajectory t: side, hit, patch point x(th, s) = base + th d1 + s d2
// (each operation rounded as written).
MS_D int traj_start(const RefArgs &a, int64_t t, int &side, int64_t &k, double y[4], const double *&patch)
{
    side = t >= a.K ? 1 : 0;
    k = t - (side ? a.K : 0);
    const double *pr = a.params + 4 * k + 2 * side;
    patch = (side ? a.Sp : a.U) + a.pstride * k;
    double th = pr[0], s = pr[1];
#pragma unroll
    for (int c = 0; c < 4; ++c) y[c] = (patch[c] + th * patch[4 + c]) + s * patch[8 + c];
    return 0;
}

MS_D bool hit_active(const RefArgs &a, int64_t k) { return a.status == nullptr || a.status[k] < 0; }

// One step of the map on the state alone.  Not inlined, so that the forward
// pass and the adjoint's recomputation of a segment run the very same code
// and reproduce the same states bit for bit.
__device__ __noinline__ d4 rk_state_step(d4 y0, const double *__restrict__ w, double h, Model md)
{
#pragma clang fp contract(fast)
    double y[4] = {y0.x, y0.y, y0.z, y0.w};
    double k[S][4];
#pragma unroll
    for (int i = 0; i < S; ++i) {
        double ys[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < i; ++j)
                if (RK_NZ[i][j]) acc += c_cv.a[i][j] * k[j][c];
            ys[c] = y[c] + h * acc;
        }
        rk_field(md, w[i], ys, k[i]);
    }
    d4 r;
    double out[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (RK_NZB[i]) acc += c_cv.b[i] * k[i][c];
        out[c] = y[c] + h * acc;
    }
    r.x = out[0]; r.y = out[1]; r.z = out[2]; r.w = out[3];
    return r;
}

// One step of the state together with one tangent column v: the variational
// equations v' = A(f, y) v (+ dF/de when `ecol`), integrated with the same
// stages, which is the exact derivative of the discrete step.
MS_D void rk_tangent_step(double y[4], double v[4], const double *__restrict__ w, const double *__restrict__ dwde,
                          double h, const Model &md, bool ecol)
{
#pragma clang fp contract(fast)
    double k[S][4], kv[S][4];
#pragma unroll
    for (int i = 0; i < S; ++i) {
        double ys[4], vs[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0, accv = 0.0;
#pragma unroll
            for (int j = 0; j < i; ++j)
                if (RK_NZ[i][j]) {
                    acc += c_cv.a[i][j] * k[j][c];
                    accv += c_cv.a[i][j] * kv[j][c];
                }
            ys[c] = y[c] + h * acc;
            vs[c] = v[c] + h * accv;
        }
        OmegaD o = omega_derivs(md, ys[0], ys[1]);
        double wi = w[i];
        k[i][0] = ys[2];
        k[i][1] = ys[3];
        k[i][2] = 2.0 * ys[3] + wi * o.Ox;
        k[i][3] = -2.0 * ys[2] + wi * o.Oy;
        kv[i][0] = vs[2];
        kv[i][1] = vs[3];
        kv[i][2] = wi * (o.Oxx * vs[0] + o.Oxy * vs[1]) + 2.0 * vs[3];
        kv[i][3] = wi * (o.Oxy * vs[0] + o.Oyy * vs[1]) - 2.0 * vs[2];
        if (ecol) {
            kv[i][2] += dwde[i] * o.Ox;
            kv[i][3] += dwde[i] * o.Oy;
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double acc = 0.0, accv = 0.0;
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (RK_NZB[i]) {
                acc += c_cv.b[i] * k[i][c];
                accv += c_cv.b[i] * kv[i][c];
            }
        y[c] = y[c] + h * acc;
        v[c] = v[c] + h * accv;
    }
}

MS_D const double *stage_row(const double *tab, int64_t s, int32_t steps)
{
    return tab + (size_t)(s % steps) * S;
}

// State pass: endpoint of every trajectory; with a.ckpt, the state before
// every ck-th step.
__global__ void __launch_bounds__(RF_BLOCK) k_ref_state(RefArgs a)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * a.K) return;
    int side;
    int64_t k;
    double y0[4];
    const double *patch;
    traj_start(a, t, side, k, y0, patch);
    if (!hit_active(a, k)) return;
    const SideMap sm = a.side[side];
    const int64_t T2 = 2 * a.K;
    d4 y{y0[0], y0[1], y0[2], y0[3]};
    for (int64_t s = 0; s < sm.nsteps; ++s) {
        if (a.ckpt && s % a.ck == 0) {
            double v[4] = {y.x, y.y, y.z, y.w};
            store_d4(a.ckpt + ((s / a.ck) * T2 + t) * 4, v);
        }
        y = rk_state_step(y, stage_row(sm.w, s, sm.steps), sm.h, a.md);
    }
    double v[4] = {y.x, y.y, y.z, y.w};
    store_d4(a.yend + 4 * t, v);
}

// Tangent pass: thread (column c, trajectory t); columns d/dth, d/ds, d/de.
__global__ void __launch_bounds__(RF_BLOCK) k_ref_tangent(RefArgs a)
{
    const int64_t T2 = 2 * a.K;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 3 * T2) return;
    int col = (int)(gid / T2);
    int64_t t = gid - col * T2;
    int side;
    int64_t k;
    double y[4];
    const double *patch;
    traj_start(a, t, side, k, y, patch);
    if (!hit_active(a, k)) return;
    const SideMap sm = a.side[side];
    double v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = col == 2 ? 0.0 : patch[4 * (col + 1) + c];
    const bool ecol = col == 2;
    for (int64_t s = 0; s < sm.nsteps; ++s)
        rk_tangent_step(y, v, stage_row(sm.w, s, sm.steps), stage_row(sm.dwde, s, sm.steps), sm.h, a.md, ecol);
    store_d4(a.dend + ((int64_t)col * T2 + t) * 4, v);
    if (col == 0) store_d4(a.yend + 4 * t, y);
}

// f, r (and J, grad = 2 J^T f in tangent mode) per hit.
__global__ void __launch_bounds__(RF_BLOCK) k_ref_combine(RefArgs a, int tangent, double *f_out, double *r_out,
                                                          double *J_out, double *g_out)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.K) return;
    const int64_t T2 = 2 * a.K;
    const double *yu = a.yend + 4 * k, *ys = a.yend + 4 * (a.K + k);
    double f[4], r = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        f[c] = yu[c] - ys[c];
        r += f[c] * f[c];
    }
    if (f_out) store_d4(f_out + 4 * k, f);
    if (r_out) r_out[k] = r;
    if (!tangent) return;
    double J[4][5];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        J[c][0] = a.dend[(0 * T2 + k) * 4 + c];
        J[c][1] = a.dend[(1 * T2 + k) * 4 + c];
        J[c][2] = -a.dend[(0 * T2 + a.K + k) * 4 + c];
        J[c][3] = -a.dend[(1 * T2 + a.K + k) * 4 + c];
        J[c][4] = a.dend[(2 * T2 + k) * 4 + c] - a.dend[(2 * T2 + a.K + k) * 4 + c];
    }
    if (J_out)
        for (int c = 0; c < 4; ++c)
            for (int j = 0; j < 5; ++j) J_out[20 * k + 5 * c + j] = J[c][j];
    if (g_out)
        for (int j = 0; j < 5; ++j) {
            double acc = 0.0;
            for (int c = 0; c < 4; ++c) acc += J[c][j] * f[c];
            g_out[5 * k + j] = 2.0 * acc;
        }
}

// The adjoint runs backwards over windows of consecutive steps (whole
// checkpoint segments).  For one window:
//   k_adj_states  per (segment, trajectory): the states before every step of
//                 the segment, recomputed from its checkpoint;
//   k_adj_jac     per (step, trajectory, column): the step's Jacobian
//                 M_n = d y_{n+1} / d y_n (columns 0-3, a tangent step from a
//                 unit vector) and d y_{n+1} / d e (column 4), all steps of the
//                 window in parallel;
//   k_adj_reverse per trajectory: lam <- M_n^T lam and ge += (d y_{n+1}/de) . lam
//                 for n from the last step of the window down to the first.
// This is the transpose of the discrete map, step by step (the discrete
// adjoint), with the sequential part reduced to 4 x 4 products.
__global__ void __launch_bounds__(RF_BLOCK) k_adj_states(RefArgs a, int64_t s_lo, int64_t s_hi, double *states)
{
    const int64_t T2 = 2 * a.K;
    const int64_t nseg = (s_hi - s_lo + a.ck - 1) / a.ck;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nseg * T2) return;
    const int64_t sg = gid / T2, t = gid - sg * T2;
    const int side = t >= a.K ? 1 : 0;
    const SideMap sm = a.side[side];
    const int64_t s0 = s_lo + sg * a.ck;
    int64_t s1 = s0 + a.ck < s_hi ? s0 + a.ck : s_hi;
    if (s1 > sm.nsteps) s1 = sm.nsteps;
    if (s0 >= s1) return;
    d4 y = load_d4(a.ckpt + ((s0 / a.ck) * T2 + t) * 4);
    for (int64_t s = s0; s < s1; ++s) {
        double v[4] = {y.x, y.y, y.z, y.w};
        store_d4(states + ((s - s_lo) * T2 + t) * 4, v);
        if (s + 1 < s1) y = rk_state_step(y, stage_row(sm.w, s, sm.steps), sm.h, a.md);
    }
}

__global__ void __launch_bounds__(RF_BLOCK) k_adj_jac(RefArgs a, int64_t s_lo, int64_t s_hi, const double *states,
                                                      double *jac)
{
    const int64_t T2 = 2 * a.K;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (s_hi - s_lo) * T2 * 5) return;
    const int64_t cell = gid / 5;
    const int col = (int)(gid - cell * 5);
    const int64_t sl = cell / T2, t = cell - sl * T2;
    const int side = t >= a.K ? 1 : 0;
    const SideMap sm = a.side[side];
    const int64_t s = s_lo + sl;
    if (s >= sm.nsteps) return;
    const d4 ys = load_d4(states + (sl * T2 + t) * 4);
    double y[4] = {ys.x, ys.y, ys.z, ys.w};
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (col < 4) v[col] = 1.0;
    rk_tangent_step(y, v, stage_row(sm.w, s, sm.steps), stage_row(sm.dwde, s, sm.steps), sm.h, a.md, col == 4);
    store_d4(jac + gid * 4, v);
}

// lam (4) and ge per trajectory live in adj[5 t ...]; init seeds lam = +-2 f.
__global__ void __launch_bounds__(RF_BLOCK) k_adj_reverse(RefArgs a, int64_t s_lo, int64_t s_hi, const double *jac,
                                                          double *adj, const double *f, int init)
{
    const int64_t T2 = 2 * a.K;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T2) return;
    const int side = t >= a.K ? 1 : 0;
    const int64_t k = t - (side ? a.K : 0);
    const SideMap sm = a.side[side];
    double lam[4], ge;
    if (init) {
        const double sg = side ? -2.0 : 2.0;
        for (int c = 0; c < 4; ++c) lam[c] = sg * f[4 * k + c];
        ge = 0.0;
    } else {
        for (int c = 0; c < 4; ++c) lam[c] = adj[5 * t + c];
        ge = adj[5 * t + 4];
    }
    const int64_t hi = s_hi < sm.nsteps ? s_hi : sm.nsteps;
    for (int64_t s = hi - 1; s >= s_lo; --s) {
        const double *J = jac + ((s - s_lo) * T2 + t) * 20;   // 5 columns of 4
        double m[5][4];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const d4 q = load_d4(J + 4 * c);
            m[c][0] = q.x; m[c][1] = q.y; m[c][2] = q.z; m[c][3] = q.w;
        }
        ge += ((m[4][0] * lam[0] + m[4][1] * lam[1]) + m[4][2] * lam[2]) + m[4][3] * lam[3];
        double nl[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) nl[c] = ((m[c][0] * lam[0] + m[c][1] * lam[1]) + m[c][2] * lam[2]) + m[c][3] * lam[3];
#pragma unroll
        for (int c = 0; c < 4; ++c) lam[c] = nl[c];
    }
    for (int c = 0; c < 4; ++c) adj[5 * t + c] = lam[c];
    adj[5 * t + 4] = ge;
}

// Per trajectory: the gradient with respect to its patch parameters
// (lam . d1, lam . d2) and its share of d r / d e.
__global__ void __launch_bounds__(RF_BLOCK) k_adj_finish(RefArgs a, const double *adj)
{
    const int64_t T2 = 2 * a.K;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T2) return;
    const int side = t >= a.K ? 1 : 0;
    const int64_t k = t - (side ? a.K : 0);
    const double *patch = (side ? a.Sp : a.U) + a.pstride * k;
    double g0 = 0.0, g1 = 0.0;
    for (int c = 0; c < 4; ++c) {
        g0 += adj[5 * t + c] * patch[4 + c];
        g1 += adj[5 * t + c] * patch[8 + c];
    }
    a.gpart[3 * t + 0] = g0;
    a.gpart[3 * t + 1] = g1;
    a.gpart[3 * t + 2] = adj[5 * t + 4];
}

__global__ void __launch_bounds__(RF_BLOCK) k_ref_grad(RefArgs a, double *g_out)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.K) return;
    const double *gu = a.gpart + 3 * k, *gs = a.gpart + 3 * (a.K + k);
    g_out[5 * k + 0] = gu[0];
    g_out[5 * k + 1] = gu[1];
    g_out[5 * k + 2] = gs[0];
    g_out[5 * k + 3] = gs[1];
    g_out[5 * k + 4] = gu[2] + gs[2];
}

// The stage values of both sides for one period (entry (n, i) at step n of
// a period, stage i), into the workspace: w, and dw/de when wanted.
struct TableArgs {
    double *w[2], *dwde[2];
    int32_t steps[2];
    double e;
};

__global__ void __launch_bounds__(256) k_ref_tables(TableArgs t)
{
    const int64_t n0 = (int64_t)t.steps[0] * S, n1 = (int64_t)t.steps[1] * S;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n0 + n1) return;
    const int sd = i >= n0;
    const int64_t k = sd ? i - n0 : i;
    const int64_t step = k / S;
    const int q = (int)(k - step * S);
    const double cf = cos(stage_abscissa(step, c_cv.c[q], t.steps[sd]));
    const double om = 1.0 / (1.0 + t.e * cf);
    t.w[sd][k] = om;
    if (t.dwde[sd]) t.dwde[sd][k] = -cf * om * om;
}

// ------------------------------------------------------------ damped Newton

__global__ void __launch_bounds__(RF_BLOCK) k_newton_init(const double *x0, NewtonState ns, int64_t K)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    newton_init(k, x0, ns);
}

// One decision per running hit after the tangent pass at its trial point q.
__global__ void __launch_bounds__(RF_BLOCK) k_newton_update(RefArgs a, NewtonState ns, NewtonCfg cfg)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.K || ns.status[k] >= 0) return;
    const int64_t T2 = 2 * a.K;
    const double *yu = a.yend + 4 * k, *ys = a.yend + 4 * (a.K + k);
    double f[4], M[4][4];
    for (int c = 0; c < 4; ++c) {
        f[c] = yu[c] - ys[c];
        M[c][0] = a.dend[(0 * T2 + k) * 4 + c];
        M[c][1] = a.dend[(1 * T2 + k) * 4 + c];
        M[c][2] = -a.dend[(0 * T2 + a.K + k) * 4 + c];
        M[c][3] = -a.dend[(1 * T2 + a.K + k) * 4 + c];
    }
    newton_decide(k, f, M, ns, cfg);
}

__global__ void __launch_bounds__(RF_BLOCK) k_newton_finish(NewtonState ns, int64_t K, double *x_out, double *f_out,
                                                            double *r_out, int32_t *st_out, int32_t *tr_out)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    newton_finish(k, ns, x_out, f_out, r_out, st_out, tr_out);
}

// ---------------------------------------------------------------- host side

struct RefLayout {
    size_t o_w[2], o_dwde[2], o_yend, o_dend, o_gpart, o_ckpt, o_states, o_jac, o_adj, o_nw, total;
    int64_t n_ck, win_steps, n_steps_max;
};

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t side_steps(const map_params_t *m)
{
    int64_t np = m->n_periods < 0 ? -(int64_t)m->n_periods : m->n_periods;
    return (int64_t)m->steps_per_period * np;
}

int check_maps(const map_params_t *fwd, const map_params_t *bwd)
{
    if (!fwd || !bwd) return fail(MS_E_ARG, "refine: NULL map parameters");
    for (const map_params_t *m : {fwd, bwd}) {
        if (m->steps_per_period <= 0) return fail(MS_E_ARG, "refine: steps_per_period must be > 0");
        if (!(m->e >= 0.0 && m->e < 1.0) || !(m->mu >= 0.0 && m->mu <= 1.0))
            return fail(MS_E_ARG, "refine: need 0 <= e < 1 and 0 <= mu <= 1");
    }
    if (fwd->mu != bwd->mu || fwd->e != bwd->e)
        return fail(MS_E_ARG, "refine: both sides must use the same mu and e");
    return MS_OK;
}

// Steps per adjoint window: whole checkpoint segments, as many as fit
// ADJ_WINDOW_BYTES of states and step Jacobians (at least one segment).
constexpr int64_t ADJ_WINDOW_BYTES = (int64_t)256 << 20;
constexpr int64_t ADJ_BYTES_PER_STEP = 32 + 5 * 32;   // per trajectory: state + 5 Jacobian columns

RefLayout ref_layout(int64_t K, const map_params_t *fwd, const map_params_t *bwd, int32_t ck, int32_t mode)
{
    RefLayout L;
    memset(&L, 0, sizeof L);
    const size_t T2 = (size_t)(2 * K);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = al256(o + (bytes ? bytes : 1)); return at; };
    const map_params_t *m[2] = {fwd, bwd};
    for (int sd = 0; sd < 2; ++sd) {
        const size_t tb = (size_t)m[sd]->steps_per_period * S * 8;
        L.o_w[sd] = take(tb);
        L.o_dwde[sd] = take(mode != MS_REFINE_RESIDUAL ? tb : 0);
    }
    L.o_yend = take(T2 * 32);
    L.o_dend = take((mode == MS_REFINE_TANGENT || mode == MS_REFINE_NEWTON) ? 3 * T2 * 32 : 0);
    L.o_gpart = take(mode == MS_REFINE_ADJOINT ? T2 * 24 : 0);
    if (mode == MS_REFINE_ADJOINT) {
        const int64_t a = side_steps(fwd), b = side_steps(bwd);
        L.n_steps_max = a > b ? a : b;
        L.n_ck = ceil_div(L.n_steps_max, ck);
        int64_t segs = ADJ_WINDOW_BYTES / ((int64_t)(T2 > 0 ? T2 : 1) * ADJ_BYTES_PER_STEP * ck);
        if (segs < 1) segs = 1;
        if (segs > L.n_ck) segs = L.n_ck > 0 ? L.n_ck : 1;
        L.win_steps = segs * ck;
        L.o_ckpt = take((size_t)L.n_ck * T2 * 32);
        L.o_states = take((size_t)L.win_steps * T2 * 32);
        L.o_jac = take((size_t)L.win_steps * T2 * 160);
        L.o_adj = take(T2 * 40);
    } else {
        L.o_ckpt = take(0);
        L.o_states = take(0);
        L.o_jac = take(0);
        L.o_adj = take(0);
    }
    L.o_nw = take(mode == MS_REFINE_NEWTON ? (size_t)K * (18 * 8 + 3 * 4) + 9 * 256 : 0);
    L.total = o;
    return L;
}

// Kernel arguments of one call, with the stage values of both sides in the
// workspace; queues the kernel that computes them.
int make_args(RefArgs &a, const double *params, int64_t K, const patch_t *U, const patch_t *Sp, int32_t stride,
              const map_params_t *fwd, const map_params_t *bwd, int32_t ck, int need_dwde, char *ws,
              const RefLayout &L, hipStream_t st)
{
    if (!cv_pattern_ok()) return fail(MS_E_ARG, "refine: internal tableau pattern mismatch");
    memset(&a, 0, sizeof a);
    a.params = params;
    a.U = (const double *)U;
    a.Sp = (const double *)Sp;
    a.K = K;
    a.pstride = stride ? 12 : 0;
    a.md = Model{fwd->mu, 1.0 - fwd->mu};
    a.ck = ck;
    const map_params_t *m[2] = {fwd, bwd};
    TableArgs t;
    t.e = fwd->e;
    for (int sd = 0; sd < 2; ++sd) {
        SideMap &sm = a.side[sd];
        t.w[sd] = (double *)(ws + L.o_w[sd]);
        t.dwde[sd] = need_dwde ? (double *)(ws + L.o_dwde[sd]) : nullptr;
        t.steps[sd] = m[sd]->steps_per_period;
        sm.w = t.w[sd];
        sm.dwde = need_dwde ? t.dwde[sd] : t.w[sd];
        sm.nsteps = side_steps(m[sd]);
        sm.steps = m[sd]->steps_per_period;
        sm.h = (m[sd]->n_periods < 0 ? -RK_TWO_PI : RK_TWO_PI) / (double)m[sd]->steps_per_period;
    }
    const int64_t n = ((int64_t)t.steps[0] + t.steps[1]) * S;
    MS_LAUNCH("k_ref_tables", k_ref_tables, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, t);
    MS_HIP(hipGetLastError());
    return MS_OK;
}

unsigned blocks_for(int64_t n) { return (unsigned)ceil_div(n > 0 ? n : 1, RF_BLOCK); }

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" int refine_workspace_size(int64_t K, const map_params_t *fwd, const map_params_t *bwd, int32_t ckpt_every,
                                     int32_t mode, size_t *bytes)
{
    if (!bytes || K < 0) return fail(MS_E_ARG, "refine_workspace_size: bad argument");
    int rc = check_maps(fwd, bwd);
    if (rc) return rc;
    if (mode < MS_REFINE_RESIDUAL || mode > MS_REFINE_NEWTON) return fail(MS_E_ARG, "refine_workspace_size: bad mode");
    if (mode == MS_REFINE_ADJOINT && ckpt_every <= 0) return fail(MS_E_ARG, "refine: ckpt_every must be > 0");
    *bytes = ref_layout(K, fwd, bwd, ckpt_every > 0 ? ckpt_every : 1, mode).total;
    return MS_OK;
}

extern "C" int refine_grad(const double *params_dev, int64_t K, const patch_t *U_dev, const patch_t *S_dev,
                           int32_t patch_stride, const map_params_t *fwd, const map_params_t *bwd, int32_t ckpt_every,
                           int32_t mode, double *f_dev, double *r_dev, double *grad_dev, double *J_dev, void *ws,
                           size_t ws_bytes, void *stream)
{
    if (K < 0 || (K > 0 && (!params_dev || !U_dev || !S_dev))) return fail(MS_E_ARG, "refine_grad: bad argument");
    if (patch_stride != 0 && patch_stride != 1) return fail(MS_E_ARG, "refine_grad: patch_stride must be 0 or 1");
    if (mode < MS_REFINE_RESIDUAL || mode > MS_REFINE_TANGENT) return fail(MS_E_ARG, "refine_grad: bad mode");
    if (mode == MS_REFINE_ADJOINT && ckpt_every <= 0) return fail(MS_E_ARG, "refine_grad: the adjoint needs ckpt_every > 0");
    if (K > ((int64_t)1 << 28)) return fail(MS_E_ARG, "refine_grad: K too large");
    int rc = check_maps(fwd, bwd);
    if (rc) return rc;
    if (K == 0) return MS_OK;
    if (mode == MS_REFINE_ADJOINT && (!f_dev || !grad_dev))
        return fail(MS_E_ARG, "refine_grad: the adjoint needs f_dev and grad_dev");
    const int32_t ck = mode == MS_REFINE_ADJOINT ? ckpt_every : 1;
    RefLayout L = ref_layout(K, fwd, bwd, ck, mode);
    if (!ws || ws_bytes < L.total) return fail(MS_E_WORKSPACE, "refine_grad: workspace too small");
    char *w = (char *)ws;
    hipStream_t st = (hipStream_t)stream;
    RefArgs a;
    if ((rc = make_args(a, params_dev, K, U_dev, S_dev, patch_stride, fwd, bwd, ck, mode != MS_REFINE_RESIDUAL, w, L,
                        st)))
        return rc;
    a.yend = (double *)(w + L.o_yend);
    a.dend = (double *)(w + L.o_dend);
    a.gpart = (double *)(w + L.o_gpart);
    const int64_t T2 = 2 * K;
    if (mode == MS_REFINE_TANGENT) {
        MS_LAUNCH("k_ref_tangent", k_ref_tangent, dim3(blocks_for(3 * T2)), dim3(RF_BLOCK), 0, st, a);
        MS_LAUNCH("k_ref_combine", k_ref_combine, dim3(blocks_for(K)), dim3(RF_BLOCK), 0, st, a, 1, f_dev, r_dev, J_dev,
                  grad_dev);
    } else {
        if (mode == MS_REFINE_ADJOINT) a.ckpt = (double *)(w + L.o_ckpt);
        MS_LAUNCH("k_ref_state", k_ref_state, dim3(blocks_for(T2)), dim3(RF_BLOCK), 0, st, a);
        MS_LAUNCH("k_ref_combine", k_ref_combine, dim3(blocks_for(K)), dim3(RF_BLOCK), 0, st, a, 0, f_dev, r_dev,
                  (double *)nullptr, (double *)nullptr);
        if (mode == MS_REFINE_ADJOINT) {
            double *states = (double *)(w + L.o_states), *jac = (double *)(w + L.o_jac), *adj = (double *)(w + L.o_adj);
            const int64_t W = L.win_steps;
            int64_t nwin = ceil_div(L.n_steps_max, W);
            if (nwin < 1) nwin = 1;
            for (int64_t wi = nwin - 1; wi >= 0; --wi) {
                const int64_t s_lo = wi * W;
                const int64_t s_hi = s_lo + W < L.n_steps_max ? s_lo + W : L.n_steps_max;
                const int64_t nseg = ceil_div(s_hi - s_lo, (int64_t)ck);
                if (s_hi > s_lo) {
                    MS_LAUNCH("k_adj_states", k_adj_states, dim3(blocks_for(nseg * T2)), dim3(RF_BLOCK), 0, st, a, s_lo,
                              s_hi, states);
                    MS_LAUNCH("k_adj_jac", k_adj_jac, dim3(blocks_for((s_hi - s_lo) * T2 * 5)), dim3(RF_BLOCK), 0, st, a,
                              s_lo, s_hi, (const double *)states, jac);
                }
                MS_LAUNCH("k_adj_reverse", k_adj_reverse, dim3(blocks_for(T2)), dim3(RF_BLOCK), 0, st, a, s_lo, s_hi,
                          (const double *)jac, adj, (const double *)f_dev, (int)(wi == nwin - 1));
            }
            MS_LAUNCH("k_adj_finish", k_adj_finish, dim3(blocks_for(T2)), dim3(RF_BLOCK), 0, st, a, (const double *)adj);
            MS_LAUNCH("k_ref_grad", k_ref_grad, dim3(blocks_for(K)), dim3(RF_BLOCK), 0, st, a, grad_dev);
        }
    }
    MS_HIP(hipGetLastError());
    return MS_OK;
}

extern "C" int refine_newton(const double *params_in_dev, double *params_out_dev, int64_t K, const patch_t *U_dev,
                             const patch_t *S_dev, int32_t patch_stride, const map_params_t *fwd,
                             const map_params_t *bwd, const newton_params_t *np, double *f_dev, double *r_dev,
                             int32_t *status_dev, int32_t *trials_dev, void *ws, size_t ws_bytes, void *stream)
{
    if (K < 0 || !np || (K > 0 && (!params_in_dev || !params_out_dev || !U_dev || !S_dev)))
        return fail(MS_E_ARG, "refine_newton: bad argument");
    if (patch_stride != 0 && patch_stride != 1) return fail(MS_E_ARG, "refine_newton: patch_stride must be 0 or 1");
    if (np->max_trials < 0 || np->max_trials > 100000) return fail(MS_E_ARG, "refine_newton: max_trials out of range");
    if (!(np->alpha0 > 0.0 && np->alpha0 <= 1.0) || !(np->alpha_min > 0.0) || !(np->tol >= 0.0))
        return fail(MS_E_ARG, "refine_newton: need 0 < alpha0 <= 1, alpha_min > 0, tol >= 0");
    if (K > ((int64_t)1 << 28)) return fail(MS_E_ARG, "refine_newton: K too large");
    int rc = check_maps(fwd, bwd);
    if (rc) return rc;
    if (K == 0) return MS_OK;
    RefLayout L = ref_layout(K, fwd, bwd, 1, MS_REFINE_NEWTON);
    if (!ws || ws_bytes < L.total) return fail(MS_E_WORKSPACE, "refine_newton: workspace too small");
    char *w = (char *)ws;
    NewtonState ns;
    {
        size_t o = L.o_nw;
        auto take = [&](size_t bytes) { size_t at = o; o = al256(o + bytes); return w + at; };
        ns.p = (double *)take((size_t)K * 32);
        ns.q = (double *)take((size_t)K * 32);
        ns.delta = (double *)take((size_t)K * 32);
        ns.fp = (double *)take((size_t)K * 32);
        ns.rp = (double *)take((size_t)K * 8);
        ns.alpha = (double *)take((size_t)K * 8);
        ns.status = (int32_t *)take((size_t)K * 4);
        ns.trials = (int32_t *)take((size_t)K * 4);
        ns.based = (int32_t *)take((size_t)K * 4);
        if ((size_t)(o) > L.total) return fail(MS_E_WORKSPACE, "refine_newton: internal layout");
    }
    hipStream_t st = (hipStream_t)stream;
    RefArgs a;
    if ((rc = make_args(a, ns.q, K, U_dev, S_dev, patch_stride, fwd, bwd, 1, 1, w, L, st))) return rc;
    a.yend = (double *)(w + L.o_yend);
    a.dend = (double *)(w + L.o_dend);
    a.status = ns.status;
    NewtonCfg cfg;
    cfg.tol2 = np->tol * np->tol;
    cfg.alpha0 = np->alpha0;
    cfg.alpha_min = np->alpha_min;
    cfg.max_trials = np->max_trials;
    const int64_t T2 = 2 * K;
    MS_LAUNCH("k_newton_init", k_newton_init, dim3(blocks_for(K)), dim3(RF_BLOCK), 0, st, params_in_dev, ns, K);
    for (int it = 0; it <= np->max_trials; ++it) {
        MS_LAUNCH("k_ref_tangent", k_ref_tangent, dim3(blocks_for(3 * T2)), dim3(RF_BLOCK), 0, st, a);
        MS_LAUNCH("k_newton_update", k_newton_update, dim3(blocks_for(K)), dim3(RF_BLOCK), 0, st, a, ns, cfg);
    }
    MS_LAUNCH("k_newton_finish", k_newton_finish, dim3(blocks_for(K)), dim3(RF_BLOCK), 0, st, ns, K, params_out_dev,
              f_dev, r_dev, status_dev, trials_dev);
    MS_HIP(hipGetLastError());
    return MS_OK;
}
