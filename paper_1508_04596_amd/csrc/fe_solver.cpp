// Host-driven solvers over the device kernels: flexible GMRES with classical
// Gram-Schmidt (two projections per basis vector, the second delayed into the
// next step) in FP64, damped Newton with the quadratic L2 line
// search (Sec. "Solving the non-linear system"), the adjoint solve, and the
// FP32-operator / FP64-residual refinement used in mixed mode.  An FP32
// preconditioner can also serve the FP64 operator (fe_solve_opts.pc_prec).
//
// The Krylov basis V, the Hessenberg matrix, the Givens rotations and every
// norm are FP64.  One Arnoldi step runs entirely on the device; the host reads
// back its dot products (2j + 9 numbers) to finish a Hessenberg column, update
// the Givens rotations and test convergence.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <vector>

#include "fe_internal.h"
#include "fe_mg.h"

using namespace fe;

namespace fe {

struct SolverWs {
    int m = 0;           // restart length the buffers were sized for
    bool mixed = false;  // FP32 copies allocated (FP32 operator or preconditioner)
    int64_t ndof = 0, nn = 0;
    double *R = nullptr, *Rh = nullptr, *R1 = nullptr, *xt = nullptr, *delta = nullptr;
    double *rhs = nullptr, *V = nullptr, *Z = nullptr, *D = nullptr, *tmp = nullptr;
    float *Z32 = nullptr, *D32 = nullptr, *x32 = nullptr;
    double *hbuf = nullptr;  // device: Gram-Schmidt products of a step | [255] cycle scale
    double *ydev = nullptr;  // device: combination coefficients
    double *hhost = nullptr; // pinned host copy of hbuf / y
    // 0-2 / 8-10: preconditioner start, operator start, operator end of even /
    // odd Arnoldi steps; 3: Gram-Schmidt end; 4-5: set-up; 6: batched job;
    // 11: a step's results copied; 12-13: the candidate-only dot pass
    hipEvent_t ev[16] = {};
    Mg *mg = nullptr;        // multigrid hierarchy (created on first use)
    fe_problem *owner = nullptr;  // allocations go through owner->alloc
};

static void free_ws(SolverWs *w)
{
    if (!w) return;
    fe_problem *p = w->owner;
    double *d[] = {w->R, w->Rh, w->R1, w->xt, w->delta, w->rhs, w->V, w->Z, w->D, w->tmp,
                   w->hbuf, w->ydev};
    for (double *q : d) dfree(p, q);
    dfree(p, w->Z32);
    dfree(p, w->D32);
    dfree(p, w->x32);
    hfree(p, w->hhost);
    mg_free(w->mg);
    for (auto &e : w->ev)
        if (e) (void)hipEventDestroy(e);
    delete w;
}

static int64_t ws_bytes(int64_t ndof, int64_t nn, int m, bool mixed)
{
    int64_t b = 0;
    b += 7 * ndof * 8;                 // R, Rh, R1, xt, delta, rhs, tmp
    b += (int64_t)(m + 1) * ndof * 8;  // V
    b += (int64_t)m * ndof * 8;        // Z (FP64; the adjoint solve always uses it)
    if (mixed) b += (int64_t)m * ndof * 4;  // Z32
    b += nn * 25 * 8;                  // D
    if (mixed) b += nn * 25 * 4 + ndof * 4;  // D32, x32
    b += 2 * 256 * 8;
    return b;
}

static int ensure_ws(fe_problem *p, int m, bool mixed)
{
    SolverWs *w = p->ws;
    if (w && w->m >= m && (w->mixed || !mixed)) return FE_OK;
    free_ws(w);
    p->ws = nullptr;
    w = new SolverWs();
    w->owner = p;
    w->m = m;
    w->mixed = mixed;
    w->ndof = p->ndof;
    w->nn = p->nn;
    const size_t nb = sizeof(double) * p->ndof;
    hipError_t e = hipSuccess;
    double **vecs[] = {&w->R, &w->Rh, &w->R1, &w->xt, &w->delta, &w->rhs, &w->tmp};
    for (double **q : vecs)
        if (e == hipSuccess) e = dalloc(p, q, nb);
    if (e == hipSuccess) e = dalloc(p, &w->V, nb * (m + 1));
    if (e == hipSuccess) e = dalloc(p, &w->Z, nb * m);
    if (e == hipSuccess && mixed) e = dalloc(p, &w->Z32, sizeof(float) * p->ndof * m);
    if (e == hipSuccess) e = dalloc(p, &w->D, sizeof(double) * 25 * p->nn);
    if (e == hipSuccess && mixed) e = dalloc(p, &w->D32, sizeof(float) * 25 * p->nn);
    if (e == hipSuccess && mixed) e = dalloc(p, &w->x32, sizeof(float) * p->ndof);
    if (e == hipSuccess) e = dalloc(p, &w->hbuf, sizeof(double) * 256);
    if (e == hipSuccess) e = dalloc(p, &w->ydev, sizeof(double) * 256);
    if (e == hipSuccess) e = halloc(p, &w->hhost, sizeof(double) * 256);
    for (auto &ev : w->ev)
        if (e == hipSuccess) e = hipEventCreate(&ev);
    if (e == hipSuccess && !p->slots25)
        e = dalloc(p, &p->slots25, (size_t)n_tiles(p->geo) * BOXN * 25 * sizeof(double));
    if (e != hipSuccess) {
        free_ws(w);
        return hip_fail(e, "hipMalloc (solver workspace)");
    }
    p->ws = w;
    return FE_OK;
}

// ||a||_2 (device reduction, host result; synchronises the stream)
static int norm2(fe_problem *p, const double *a, hipStream_t st, double *out)
{
    FE_CHECK_HIP(launch_norm2_partial(a, p->ndof, p->partial, st));
    FE_CHECK_HIP(launch_reduce(p->partial, 1, p->scal, nullptr, true, st, red_blocks(p->ndof)));
    FE_CHECK_HIP(hipMemcpyAsync(p->ws->hhost, p->scal, sizeof(double), hipMemcpyDeviceToHost, st));
    FE_CHECK_HIP(hipStreamSynchronize(st));
    *out = p->ws->hhost[0];
    return FE_OK;
}

// Linear operator / preconditioner callbacks for one FGMRES solve.
struct LinSys {
    // z_j = M v_j (v FP64, z in the Krylov-vector type of the solve)
    std::function<hipError_t(const double *v, void *z)> prec;
    // w = A z (z in the Krylov-vector type), w FP64
    std::function<hipError_t(const void *z, double *w)> op_z;
    // w = A x with x FP64 (true residual)
    std::function<hipError_t(const double *x, double *w)> op64;
    bool z32 = false;   // Krylov vectors z_j stored in FP32
    bool op32 = false;  // FP32 operator: every cycle ends with the FP64 true residual
};

struct LinStats {
    int its = 0;
    bool converged = false;
    double t_jv = 0, t_prec = 0, t_orth = 0;
    double res_true = 0;
};

// Column c of the Hessenberg matrix H (m columns, entries 0 .. c+1 set) gets
// the rotations 0 .. c-1, defines rotation c and advances g; returns the
// residual estimate |g[c+1]|.
double givens_column(std::vector<double> &H, int m, int c, std::vector<double> &cs,
                     std::vector<double> &sn, std::vector<double> &g)
{
    for (int i = 0; i < c; ++i) {
        const double a = H[(size_t)i * m + c], b = H[(size_t)(i + 1) * m + c];
        H[(size_t)i * m + c] = cs[i] * a + sn[i] * b;
        H[(size_t)(i + 1) * m + c] = -sn[i] * a + cs[i] * b;
    }
    const double a = H[(size_t)c * m + c], hn = H[(size_t)(c + 1) * m + c];
    const double den = std::hypot(a, hn);
    if (den == 0.0) {
        cs[c] = 1.0;
        sn[c] = 0.0;
    } else {
        cs[c] = a / den;
        sn[c] = hn / den;
    }
    H[(size_t)c * m + c] = cs[c] * a + sn[c] * hn;
    H[(size_t)(c + 1) * m + c] = 0.0;
    g[c + 1] = -sn[c] * g[c];
    g[c] = cs[c] * g[c];
    return std::fabs(g[c + 1]);
}

// The residual estimate that column c with entries col[0 .. c+1] would give,
// state unchanged.
double givens_estimate(const std::vector<double> &col, int c, const std::vector<double> &cs,
                       const std::vector<double> &sn, const std::vector<double> &g)
{
    std::vector<double> v(col.begin(), col.begin() + c + 2);
    for (int i = 0; i < c; ++i) {
        const double a = v[i], b = v[i + 1];
        v[i] = cs[i] * a + sn[i] * b;
        v[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double den = std::hypot(v[c], v[c + 1]);
    return den == 0.0 ? std::fabs(g[c]) : std::fabs(g[c]) * std::fabs(v[c + 1]) / den;
}

// Solve A x = b for x (x = 0 on entry) to |b - A x| <= rtol |b|, FGMRES(m).
// Mixed mode (op32): the Arnoldi process uses the FP32 operator; each cycle
// ends with the true FP64 residual b - A x, and cycles continue while it is
// above the target, at most n_refine cycles beyond the first convergence.
// With an FP32 preconditioner and the FP64 operator (z32 without op32) only
// the storage of z_j differs from an FP64 solve (the operator widens it).
//
// Orthogonalisation is classical Gram-Schmidt with two projections per basis
// vector, the second one delayed by a step (launch_dgs_step): step j
// preconditions the candidate c_j (the previous Krylov vector after its first
// projection, divided by that vector's norm omega_j), and the same pass over
// the basis that projects the new Krylov vector also gives the candidate's
// second projection.  So column j - 1 of H is final only in step j:
// A z_{j-1} = sum_{i<j} Hp_i q_i + omega_j c_j with c_j = sum_{i<j} s_i q_i +
// sigma_j q_j gives H_{i,j-1} = Hp_i + omega_j s_i and H_{j,j-1} = omega_j
// sigma_j.  Before each step the residual that the provisional column would
// give (subdiagonal omega_j |c_j|) is checked; when it reaches the target, the
// column is finished from the candidate's dot products alone
// (launch_dgs_final), so the cycle does not pay for a step it does not use.
// The next step's preconditioner and operator act on the candidate that the
// update pass leaves on the device, so while the residual is far above the
// target (SPEC_MARGIN) they are enqueued before the host waits for the step's
// results, and the GPU does not idle during the host's Givens update.
static int fgmres(fe_problem *p, const LinSys &L, const double *b, double *x, double rtol, int m,
                  int max_its, int n_refine, hipStream_t st, LinStats *stats, int verbose)
{
    SolverWs *w = p->ws;
    const int64_t n = p->ndof;
    const int64_t ld = n;
    FE_CHECK_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, st));
    double beta0;
    int rc = norm2(p, b, st, &beta0);
    if (rc) return rc;
    if (!std::isfinite(beta0)) {
        set_error("non-finite right-hand side in FGMRES");
        return FE_ENAN;
    }
    stats->its = 0;
    stats->converged = false;
    if (beta0 == 0.0) {
        stats->converged = true;
        return FE_OK;
    }
    const double target = rtol * beta0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), Hp(m + 2);
    const double *r = b;  // residual of the current cycle (b on the first cycle)
    double beta = beta0;
    int refine_left = n_refine;
    constexpr double SPEC_MARGIN = 100.0;
    while (true) {
        // candidate c_0 = r / beta (r = beta c_0)
        w->hhost[200] = beta;
        FE_CHECK_HIP(hipMemcpyAsync(w->hbuf + 255, w->hhost + 200, sizeof(double),
                                    hipMemcpyHostToDevice, st));
        FE_CHECK_HIP(launch_scale_div(n, r, w->hbuf + 255, w->V, st));
        std::fill(g.begin(), g.end(), 0.0);
        double om = beta, c2 = 1.0;  // scale and squared norm of the candidate
        double res = beta;
        bool breakdown = false;
        int kk = 0;               // final columns of H
        bool col_final = false;   // column j - 1 was finished before step j
        bool spec = false;        // step j's preconditioner and operator are enqueued
        // z_j = M c_j and w = A z_j into column j + 1, between the step's events
        auto step_events = [&](int jj) { return w->ev + ((jj & 1) ? 8 : 0); };
        auto enqueue_step = [&](int jj) -> hipError_t {
            hipEvent_t *Ej = step_events(jj);
            void *zj = L.z32 ? (void *)(w->Z32 + (int64_t)jj * ld) : (void *)(w->Z + (int64_t)jj * ld);
            hipError_t e;
            if ((e = hipEventRecord(Ej[0], st)) != hipSuccess) return e;
            if ((e = L.prec(w->V + (int64_t)jj * ld, zj)) != hipSuccess) return e;
            if ((e = hipEventRecord(Ej[1], st)) != hipSuccess) return e;
            if ((e = L.op_z(zj, w->V + (int64_t)(jj + 1) * ld)) != hipSuccess) return e;
            return hipEventRecord(Ej[2], st);
        };
        // column j - 1 of H from its provisional entries Hp and the candidate's
        // dot products s (host copy) and remaining norm sig
        auto finish = [&](int j, const double *s, double sig) {
            for (int i = 0; i < j; ++i) H[(size_t)i * m + (j - 1)] = Hp[i] + om * s[i];
            H[(size_t)j * m + (j - 1)] = om * sig;
            res = givens_column(H, m, j - 1, cs, sn, g);
            kk = j;
            if (!(om * sig > 1e-300 * beta0)) breakdown = true;
        };
        for (int j = 0;; ++j) {
            if (j >= 1) {
                bool fin = j == m || stats->its >= max_its;
                if (!fin) {
                    Hp[j] = om * std::sqrt(std::max(c2, 0.0));
                    fin = givens_estimate(Hp, j - 1, cs, sn, g) <= target;
                }
                if (fin) {
                    FE_CHECK_HIP(hipEventRecord(w->ev[12], st));
                    FE_CHECK_HIP(launch_dgs_final(w->V, ld, j, n, w->hbuf, p->partial, st));
                    FE_CHECK_HIP(hipEventRecord(w->ev[13], st));
                    FE_CHECK_HIP(hipMemcpyAsync(w->hhost, w->hbuf, sizeof(double) * (j + 1),
                                                hipMemcpyDeviceToHost, st));
                    FE_CHECK_HIP(hipStreamSynchronize(st));
                    float ms;
                    if (hipEventElapsedTime(&ms, w->ev[12], w->ev[13]) == hipSuccess) stats->t_orth += ms * 1e-3;
                    const double *hh = w->hhost;
                    double ss = 0.0;
                    for (int i = 0; i < j; ++i) ss += hh[i] * hh[i];
                    const double s2 = hh[j] - ss;
                    if (!std::isfinite(s2)) {
                        set_error("non-finite Krylov norm");
                        return FE_ENAN;
                    }
                    finish(j, hh, s2 > 0.0 ? std::sqrt(s2) : 0.0);
                    if (res <= target || stats->its >= max_its || j == m || breakdown) break;
                    // the estimate was optimistic: take step j, whose dot pass
                    // must not finish column j - 1 (and rotate g) a second time
                    col_final = true;
                }
            } else if (stats->its >= max_its) {
                break;
            }
            // Arnoldi step j: z_j = M c_j, w = A z_j into column j + 1 (unless
            // enqueued ahead), then the two Gram-Schmidt passes
            hipEvent_t *E = step_events(j);
            if (!spec) FE_CHECK_HIP(enqueue_step(j));
            spec = false;
            FE_CHECK_HIP(launch_dgs_step(w->V, ld, j, n, w->hbuf, p->partial, st));
            FE_CHECK_HIP(hipEventRecord(w->ev[3], st));
            FE_CHECK_HIP(hipMemcpyAsync(w->hhost, w->hbuf, sizeof(double) * (2 * j + 9),
                                        hipMemcpyDeviceToHost, st));
            FE_CHECK_HIP(hipEventRecord(w->ev[11], st));
            if (res > SPEC_MARGIN * target && j + 1 < m && stats->its + 1 < max_its) {
                FE_CHECK_HIP(enqueue_step(j + 1));
                spec = true;
            }
            FE_CHECK_HIP(hipEventSynchronize(w->ev[11]));
            stats->its++;
            float ms;
            if (hipEventElapsedTime(&ms, E[0], E[1]) == hipSuccess) stats->t_prec += ms * 1e-3;
            if (hipEventElapsedTime(&ms, E[1], E[2]) == hipSuccess) stats->t_jv += ms * 1e-3;
            if (hipEventElapsedTime(&ms, E[2], w->ev[3]) == hipSuccess) stats->t_orth += ms * 1e-3;
            const double *hh = w->hhost;
            const double sig = hh[2 * j + 3], hj = hh[2 * j + 4], omn = hh[2 * j + 5];
            const double cn2 = hh[2 * j + 8];
            if (!std::isfinite(sig) || !std::isfinite(hj) || !std::isfinite(omn) || !std::isfinite(cn2)) {
                set_error("non-finite Krylov norm");
                return FE_ENAN;
            }
            if (j == 0) {
                g[0] = om * sig;  // r = beta sigma_0 q_0
                if (!(sig > 0.0)) breakdown = true;
            } else if (!col_final) {
                finish(j, hh, sig);
            }
            col_final = false;
            // a column that already meets the target ends the cycle; the step's
            // Krylov vector is then not used
            if (breakdown || (j >= 1 && res <= target)) break;
            // provisional column j: the coefficients of w's first projection
            for (int i = 0; i < j; ++i) Hp[i] = hh[j + 1 + i];
            Hp[j] = hj;
            om = omn;
            c2 = cn2;
        }
        // y = H^{-1} g (upper triangular kk x kk), x += Z y
        for (int i = kk - 1; i >= 0; --i) {
            double s = g[i];
            for (int c = i + 1; c < kk; ++c) s -= H[(size_t)i * m + c] * y[c];
            y[i] = s / H[(size_t)i * m + i];
        }
        std::memcpy(w->hhost, y.data(), sizeof(double) * kk);
        FE_CHECK_HIP(hipMemcpyAsync(w->ydev, w->hhost, sizeof(double) * kk, hipMemcpyHostToDevice, st));
        if (L.z32)
            FE_CHECK_HIP(launch_combine<float>(w->Z32, ld, kk, w->ydev, x, n, st));
        else
            FE_CHECK_HIP(launch_combine<double>(w->Z, ld, kk, w->ydev, x, n, st));
        const bool est_conv = res <= target;
        const bool need_true = L.op32 || !est_conv;
        if (stats->its >= max_its && !est_conv) break;
        if (!need_true) {
            stats->converged = true;
            stats->res_true = res;
            break;
        }
        // true residual r = b - A x (FP64 operator)
        FE_CHECK_HIP(L.op64(x, w->tmp));
        FE_CHECK_HIP(launch_axpby(n, 1.0, b, -1.0, w->tmp, st));
        rc = norm2(p, w->tmp, st, &beta);
        if (rc) return rc;
        stats->res_true = beta;
        if (verbose > 1)
            fprintf(stderr, "  fgmres cycle: its %d est %.3e true %.3e target %.3e\n", stats->its,
                    res / beta0, beta / beta0, rtol);
        if (beta <= target) {
            stats->converged = true;
            break;
        }
        if (est_conv) {
            if (refine_left-- <= 0) break;
        }
        if (stats->its >= max_its || breakdown) break;
        // next cycle solves A d = r and adds d to x: keep x, restart from r
        // (x accumulates across cycles since each cycle adds Z y to it)
        r = w->tmp;
        // r lives in tmp; the next cycle's c_0 = r / beta copies it into V before
        // tmp is reused for the following true residual.
    }
    return FE_OK;
}

}  // namespace fe

extern "C" {

void fe_free_solver_ws(fe_problem *p)
{
    if (p && p->ws) {
        free_ws(p->ws);
        p->ws = nullptr;
    }
}

void fe_solve_opts_default(fe_solve_opts *o)
{
    if (!o) return;
    o->rtol_newton = 1e-8;
    o->rtol_lin = 1e-5;
    o->max_newton = 50;
    o->restart = 60;
    o->max_lin = 3000;
    o->n_refine = 3;
    o->krylov_op_prec = FE_FP64;
    o->ls_lambda_min = 0.05;
    o->verbose = 0;
    o->precond = FE_PC_AUTO;
    o->mg_nu = 2;
    o->mg_omega = 0.6;
    o->atol_newton = 0.0;
    o->ramp_steps = 0;
    o->mg_assembled_nodes = -1;
    o->mg_nu_post = 1;
    o->pc_prec = FE_FP64;
    o->mg_coarse_reuse = 2;
}

static bool valid_prec(fe_prec q) { return q == FE_FP64 || q == FE_FP32; }

// Resolve the preconditioner choice and make the multigrid hierarchy ready.
static int choose_precond(fe_problem *p, const fe_solve_opts &o, bool mixed, int *pc)
{
    int want = o.precond;
    if (want == FE_PC_AUTO) want = mg_num_levels(p->grid) >= 2 ? FE_PC_MULTIGRID : FE_PC_BJACOBI;
    if (want != FE_PC_MULTIGRID && want != FE_PC_BJACOBI) {
        set_error("unknown preconditioner");
        return FE_EINVAL;
    }
    *pc = want;
    if (want == FE_PC_MULTIGRID) {
        SolverWs *w = p->ws;
        const int64_t asm_nodes = mg_asm_nodes(o.mg_assembled_nodes);
        if (w->mg && ((mixed && !w->mg->mixed) || w->mg->asm_nodes != asm_nodes)) {
            mg_free(w->mg);
            w->mg = nullptr;
        }
        if (!w->mg) {
            int rc = mg_create(p, mixed, asm_nodes, &w->mg);
            if (rc) return rc;
        }
        w->mg->nu1 = o.mg_nu < 1 ? 1 : o.mg_nu;
        w->mg->nu2 = o.mg_nu_post < 0 ? w->mg->nu1 : o.mg_nu_post;
        w->mg->omega = o.mg_omega;
    }
    return FE_OK;
}

int64_t fe_solve_footprint_bytes(const fe_grid *grid, const fe_solve_opts *opts)
{
    if (!grid || grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return -1;
    fe_solve_opts d;
    fe_solve_opts_default(&d);
    if (!opts) opts = &d;
    // FP32 copies for an FP32 operator or preconditioner
    const bool mixed = opts->krylov_op_prec == FE_FP32 || opts->pc_prec == FE_FP32;
    const int64_t nn = (int64_t)(grid->nx + 1) * (grid->ny + 1) * (grid->nz + 1);
    const int64_t ndof = NF * nn;
    const int64_t ntile = (int64_t)((grid->nx + TX - 1) / TX) * ((grid->ny + TY - 1) / TY) *
                          ((grid->nz + TZ - 1) / TZ);
    auto r = [](int64_t b) { return (b + 255) / 256 * 256; };
    int64_t b = 0;
    // problem handle
    b += r(nn) + r(ndof) + r(ntile * BOXN * NF * 8) + r((int64_t)PARTIAL_COLS * RED_BLOCKS * 8) + r(256 * 8);
    // solver workspace
    b += 7 * r(8 * ndof) + r(8 * ndof * (opts->restart + 1)) + r(8 * ndof * opts->restart);
    if (mixed) b += r(4 * ndof * opts->restart) + r(4 * 25 * nn) + r(4 * ndof);
    b += r(8 * 25 * nn) + 2 * r(256 * 8) + r(ntile * BOXN * 25 * 8);
    // multigrid hierarchy
    const bool mg = opts->precond == FE_PC_MULTIGRID ||
                    (opts->precond == FE_PC_AUTO && mg_num_levels(*grid) >= 2);
    if (mg) b += mg_footprint_bytes(*grid, mixed, mg_asm_nodes(opts->mg_assembled_nodes));
    // heat-source ramping keeps the initial vector and a scaled source
    if (opts->ramp_steps > 0) b += r(8 * ndof) + r(8 * ((int64_t)grid->nx * grid->ny * grid->nz));
    return b;
}

static void fill_report(fe_solve_report *rep, const fe_solve_report &r)
{
    if (rep) *rep = r;
}

// One damped Newton solve from x (the body of newton_solve without recovery).
static int newton_core(fe_problem *p, const double *gamma, const double *s_elem, double *x,
                       const fe_solve_opts &opts, fe_solve_report *report, hipStream_t st)
{
    auto t0 = std::chrono::steady_clock::now();
    const bool mixed = opts.krylov_op_prec == FE_FP32;        // FP32 operator (GMRES-IR)
    const bool pc32 = mixed || opts.pc_prec == FE_FP32;       // FP32 preconditioner
    int rc = ensure_ws(p, opts.restart, pc32);
    if (rc) return rc;
    SolverWs *w = p->ws;
    int pc = FE_PC_BJACOBI;
    rc = choose_precond(p, opts, pc32, &pc);
    if (rc) return rc;
    if (pc == FE_PC_MULTIGRID) {
        rc = mg_set_design(w->mg, p, gamma, s_elem, st);
        if (rc) return rc;
    }
    const int64_t n = p->ndof;
    fe_solve_report rep;
    std::memset(&rep, 0, sizeof(rep));

    double *R = w->R, *Rh = w->Rh, *R1 = w->R1;
    FE_CHECK_HIP((launch_elem<double, double>(OP_RES, p->geo, x, (const double *)nullptr, gamma,
                                              s_elem, p->nmask, R, p->slots, st)));
    double r0, rn;
    double rn_before = 0.0;  // |R| before the last Newton step
    rc = norm2(p, R, st, &r0);
    if (rc) return rc;
    rep.res0 = r0;
    rep.res_hist[0] = r0;
    if (!std::isfinite(r0)) {
        set_error("non-finite initial residual");
        rep.status = FE_ENAN;
        fill_report(report, rep);
        return FE_ENAN;
    }
    rn = r0;
    LinSys L;
    L.z32 = pc32;
    L.op32 = mixed;
    L.prec = [&](const double *v, void *z) -> hipError_t {
        if (pc == FE_PC_MULTIGRID) {
            int r = pc32 ? mg_apply32(w->mg, v, (float *)z, false, st)
                         : mg_apply64(w->mg, v, (double *)z, false, st);
            return r == FE_OK ? hipSuccess : hipErrorUnknown;
        }
        if (pc32)
            return launch_block_apply<float, double, float>(w->D32, v, (float *)z, p->nn, false,
                                                            nullptr, st);
        return launch_block_apply<double, double, double>(w->D, v, (double *)z, p->nn, false,
                                                          nullptr, st);
    };
    L.op_z = [&](const void *z, double *out) -> hipError_t {
        if (mixed)
            return launch_elem<float, double>(OP_JV, p->geo, w->x32, (const float *)z, gamma,
                                              s_elem, p->nmask, out, p->slots, st);
        if (pc32)  // FP32 z_j, widened as the FP64 operator stages it
            return launch_elem_dir32(OP_JV, p->geo, x, (const float *)z, gamma, s_elem, p->nmask,
                                     out, p->slots, st);
        return launch_elem<double, double>(OP_JV, p->geo, x, (const double *)z, gamma, s_elem,
                                           p->nmask, out, p->slots, st);
    };
    L.op64 = [&](const double *v, double *out) -> hipError_t {
        return launch_elem<double, double>(OP_JV, p->geo, x, v, gamma, s_elem, p->nmask, out,
                                           p->slots, st);
    };
    int status = FE_NOT_CONVERGED;
    double lam = 1.0;
    while (true) {
        if (rn <= opts.rtol_newton * r0 || rn <= opts.atol_newton) {
            status = FE_OK;
            break;
        }
        if (rep.newton_its >= opts.max_newton) break;
        const double rn_step = rn;  // |R| at the start of this Newton step
        hipEvent_t e0 = w->ev[4], e1 = w->ev[5];
        FE_CHECK_HIP(hipEventRecord(e0, st));
        // once Newton converges fast (the last step cut |R| at least 100-fold:
        // the state now changes little) the coarsest factorisation is kept, or
        // with mg_coarse_reuse = 2 the whole preconditioner set-up
        const bool fast = rep.newton_its > 0 && rn <= 0.01 * rn_before;
        const bool keep_all = opts.mg_coarse_reuse >= 2 && fast;
        // the multigrid's coarsest-level work starts first, so that its host
        // factorisation overlaps the block diagonals below
        if (pc == FE_PC_MULTIGRID && !keep_all) {
            w->mg->reuse_coarse = opts.mg_coarse_reuse != 0 && fast;
            rc = mg_setup_begin(w->mg, p, x, st);
            if (rc) {
                rep.status = rc;
                fill_report(report, rep);
                return rc;
            }
        }
        // the FP32 state is refreshed every step: the FP32 operator of mixed
        // mode reads it
        if (pc32) FE_CHECK_HIP((launch_cast<double, float>(x, w->x32, n, st)));
        if (!keep_all && pc32) {
            // the FP32 preconditioner uses FP32 blocks only: they are formed and
            // inverted in FP32 from the FP32 state
            FE_CHECK_HIP((launch_blockdiag<float>(p->geo, w->x32, gamma, s_elem, p->nmask, w->D32,
                                                  reinterpret_cast<float *>(p->slots25), st)));
            FE_CHECK_HIP(launch_invert_blocks32(w->D32, p->nn, st));
        } else if (!keep_all) {
            FE_CHECK_HIP((launch_blockdiag<double>(p->geo, x, gamma, s_elem, p->nmask, w->D,
                                                   p->slots25, st)));
            FE_CHECK_HIP(launch_invert_blocks(w->D, nullptr, p->nn, st));
        }
        if (pc == FE_PC_MULTIGRID && !keep_all) {
            rc = mg_setup_finish(w->mg, p, w->D, pc32 ? w->D32 : nullptr,
                                 pc32 ? w->x32 : nullptr, st);
            if (rc) {
                rep.status = rc;
                fill_report(report, rep);
                return rc;
            }
        }
        FE_CHECK_HIP(launch_axpby(n, -1.0, R, 0.0, w->rhs, st));
        FE_CHECK_HIP(hipEventRecord(e1, st));
        LinStats ls;
        if (p->batch && pc == FE_PC_MULTIGRID && opts.restart <= 64) {
            BJob job;
            job.p = p;
            job.mg = w->mg;
            job.mixed = mixed;
            job.pc32 = pc32 && !mixed;
            job.b = w->rhs;
            job.x = w->delta;
            job.xlin = x;
            job.x32 = w->x32;
            job.gamma = gamma;
            job.s = s_elem;
            job.V = w->V;
            job.Z = w->Z;
            job.Z32 = w->Z32;
            job.tmp = w->tmp;
            job.partial = p->partial;
            job.n = n;
            job.m = opts.restart;
            job.max_its = opts.max_lin;
            job.n_refine = mixed ? opts.n_refine : 0;
            job.rtol = opts.rtol_lin;
            job.ready = w->ev[6];
            rc = batch_fgmres(p->batch, &job, st);
            ls.its = job.its;
            ls.converged = job.converged;
            ls.res_true = job.res_true;
        } else {
            rc = fgmres(p, L, w->rhs, w->delta, opts.rtol_lin, opts.restart, opts.max_lin,
                        mixed ? opts.n_refine : 0, st, &ls, opts.verbose);
        }
        if (rc) {
            rep.status = rc;
            fill_report(report, rep);
            return rc;
        }
        float ms;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) rep.t_setup_s += ms * 1e-3;
        rep.t_jv_s += ls.t_jv;
        rep.t_prec_s += ls.t_prec;
        rep.t_orth_s += ls.t_orth;
        if (rep.newton_its < 64) rep.lin_its[rep.newton_its] = ls.its;
        rep.lin_its_total += ls.its;
        // line search on phi(l) = |R(x + l delta)|^2 at l = 1/2 and 1
        FE_CHECK_HIP(hipEventRecord(e0, st));
        double nh, n1;
        FE_CHECK_HIP(launch_xpld(n, x, 0.5, w->delta, w->xt, st));
        FE_CHECK_HIP((launch_elem<double, double>(OP_RES, p->geo, w->xt, (const double *)nullptr,
                                                  gamma, s_elem, p->nmask, Rh, p->slots, st)));
        rc = norm2(p, Rh, st, &nh);
        if (rc) return rc;
        FE_CHECK_HIP(launch_xpld(n, x, 1.0, w->delta, w->xt, st));
        FE_CHECK_HIP((launch_elem<double, double>(OP_RES, p->geo, w->xt, (const double *)nullptr,
                                                  gamma, s_elem, p->nmask, R1, p->slots, st)));
        rc = norm2(p, R1, st, &n1);
        if (rc) return rc;
        const double phi0 = rn * rn, phih = nh * nh, phi1 = n1 * n1;
        if (!std::isfinite(phih) && !std::isfinite(phi1)) {
            set_error("non-finite residual in the line search");
            rep.status = FE_ENAN;
            fill_report(report, rep);
            return FE_ENAN;
        }
        if (!std::isfinite(phi1))
            lam = 0.5;
        else if (!std::isfinite(phih))
            lam = 1.0;
        else
            lam = fe_line_search_lambda(phi0, phih, phi1, opts.ls_lambda_min);
        if (lam == 1.0) {
            FE_CHECK_HIP(hipMemcpyAsync(x, w->xt, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
            std::swap(R, R1);
            rn = n1;
        } else if (lam == 0.5) {
            FE_CHECK_HIP(launch_xpld(n, x, 0.5, w->delta, x, st));
            std::swap(R, Rh);
            rn = nh;
        } else {
            FE_CHECK_HIP(launch_xpld(n, x, lam, w->delta, x, st));
            FE_CHECK_HIP((launch_elem<double, double>(OP_RES, p->geo, x, (const double *)nullptr,
                                                      gamma, s_elem, p->nmask, R, p->slots, st)));
            rc = norm2(p, R, st, &rn);
            if (rc) return rc;
        }
        FE_CHECK_HIP(hipEventRecord(e1, st));
        FE_CHECK_HIP(hipEventSynchronize(e1));
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) rep.t_res_s += ms * 1e-3;
        rep.newton_its++;
        if (rep.newton_its <= 64) rep.res_hist[rep.newton_its] = rn;
        rn_before = rn_step;
        rep.lambda_last = lam;
        if (opts.verbose)
            fprintf(stderr, "newton %2d  |R| %.6e  rel %.3e  lambda %.3f  lin_its %d%s\n",
                    rep.newton_its, rn, rn / r0, lam, ls.its, ls.converged ? "" : " (lin not conv)");
        if (!std::isfinite(rn)) {
            set_error("non-finite residual");
            rep.status = FE_ENAN;
            fill_report(report, rep);
            return FE_ENAN;
        }
    }
    // keep the buffer rotation consistent for the next call
    w->R = R;
    w->Rh = Rh;
    w->R1 = R1;
    FE_CHECK_HIP(hipStreamSynchronize(st));
    rep.res_final = rn;
    rep.status = status;
    rep.precond = pc;
    rep.mg_levels = pc == FE_PC_MULTIGRID ? (int)w->mg->lev.size() : 0;
    rep.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_report(report, rep);
    if (status != FE_OK) set_error("newton_solve: not converged within max_newton");
    return status;
}

int newton_solve(fe_problem *p, const double *gamma, const double *s_elem, double *x,
                 const fe_solve_opts *opts_in, fe_solve_report *report, hipStream_t st)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!p || !gamma || !s_elem || !x) {
        set_error("newton_solve: NULL argument");
        return FE_EINVAL;
    }
    fe_solve_opts opts;
    fe_solve_opts_default(&opts);
    if (opts_in) opts = *opts_in;
    if (opts.restart < 1 || opts.restart > 64 || opts.max_newton < 0 || opts.max_lin < 1 ||
        !(opts.rtol_newton >= 0) || !(opts.rtol_lin > 0) || opts.ramp_steps < 0 ||
        opts.ramp_steps > 64 || !valid_prec(opts.krylov_op_prec) || !valid_prec(opts.pc_prec)) {
        set_error("newton_solve: invalid options (restart 1..64, max_lin >= 1, rtol_lin > 0, "
                  "ramp_steps 0..64, krylov_op_prec and pc_prec FE_FP64 or FE_FP32)");
        return FE_EINVAL;
    }
    if (opts.ramp_steps == 0) return newton_core(p, gamma, s_elem, x, opts, report, st);

    // keep the initial vector: the ramp restarts from it
    const int64_t n = p->ndof;
    double *x0 = nullptr, *sk = nullptr;
    hipError_t e = dalloc(p, &x0, sizeof(double) * n);
    if (e == hipSuccess) e = dalloc(p, &sk, sizeof(double) * p->ne);
    if (e == hipSuccess) e = hipMemcpyAsync(x0, x, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
        dfree(p, x0);
        dfree(p, sk);
        return hip_fail(e, "newton_solve (ramp buffers)");
    }
    fe_solve_report r1;
    std::memset(&r1, 0, sizeof(r1));
    int rc = newton_core(p, gamma, s_elem, x, opts, &r1, st);
    if ((rc != FE_NOT_CONVERGED && rc != FE_ENAN) || !std::isfinite(r1.res0)) {
        dfree(p, x0);
        dfree(p, sk);
        r1.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        fill_report(report, r1);
        return rc;
    }
    // ramping: stage k solves with s * k / K from the previous stage's result;
    // the last stage is held to the original target rtol_newton * |R(x0)|
    fe_solve_report tot = r1;
    const double target = opts.rtol_newton * r1.res0;
    e = hipMemcpyAsync(x, x0, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
    const int K = opts.ramp_steps;
    for (int k = 1; k <= K && e == hipSuccess; ++k) {
        const double *sk_use = s_elem;
        if (k < K) {
            e = launch_axpby(p->ne, (double)k / K, s_elem, 0.0, sk, st);
            if (e != hipSuccess) break;
            sk_use = sk;
        }
        fe_solve_opts ok = opts;
        if (k == K) ok.atol_newton = std::max(opts.atol_newton, target);
        fe_solve_report rk;
        std::memset(&rk, 0, sizeof(rk));
        rc = newton_core(p, gamma, sk_use, x, ok, &rk, st);
        for (int i = 0; i < rk.newton_its && tot.newton_its + i < 64; ++i)
            tot.lin_its[tot.newton_its + i] = rk.lin_its[i];
        for (int i = 1; i <= rk.newton_its && tot.newton_its + i <= 64; ++i)
            tot.res_hist[tot.newton_its + i] = rk.res_hist[i];
        tot.newton_its += rk.newton_its;
        tot.lin_its_total += rk.lin_its_total;
        tot.t_jv_s += rk.t_jv_s;
        tot.t_prec_s += rk.t_prec_s;
        tot.t_orth_s += rk.t_orth_s;
        tot.t_res_s += rk.t_res_s;
        tot.t_setup_s += rk.t_setup_s;
        tot.res_final = rk.res_final;
        tot.lambda_last = rk.lambda_last;
        tot.ramp_stages = k;
        if (rc != FE_OK) break;
    }
    dfree(p, x0);
    dfree(p, sk);
    if (e != hipSuccess) return hip_fail(e, "newton_solve (ramp)");
    tot.status = rc;
    tot.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_report(report, tot);
    if (rc == FE_NOT_CONVERGED) set_error("newton_solve: not converged after heat-source ramping");
    return rc;
}

int fe_adjoint_solve(fe_problem *p, const double *x, const double *gamma, const double *s_elem,
                     const double *rhs, double *lambda, const fe_solve_opts *opts_in,
                     fe_solve_report *report, hipStream_t st)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!p || !x || !gamma || !s_elem || !rhs || !lambda) {
        set_error("fe_adjoint_solve: NULL argument");
        return FE_EINVAL;
    }
    fe_solve_opts opts;
    fe_solve_opts_default(&opts);
    if (opts_in) opts = *opts_in;
    if (opts.restart < 1 || opts.restart > 64 || opts.max_lin < 1 || !(opts.rtol_lin > 0) ||
        !valid_prec(opts.pc_prec)) {
        set_error("fe_adjoint_solve: invalid options (restart 1..64, max_lin >= 1, rtol_lin > 0, "
                  "pc_prec FE_FP64 or FE_FP32)");
        return FE_EINVAL;
    }
    // the operator is always FP64 here; pc_prec selects the preconditioner's
    // precision (krylov_op_prec does not apply)
    const bool pc32 = opts.pc_prec == FE_FP32;
    int rc = ensure_ws(p, opts.restart, pc32);
    if (rc) return rc;
    SolverWs *w = p->ws;
    fe_solve_report rep;
    std::memset(&rep, 0, sizeof(rep));
    int pc = FE_PC_BJACOBI;
    rc = choose_precond(p, opts, pc32, &pc);
    if (rc) return rc;
    if (pc == FE_PC_MULTIGRID) {
        rc = mg_set_design(w->mg, p, gamma, s_elem, st);
        w->mg->reuse_coarse = false;
        if (rc == FE_OK) rc = mg_setup_begin(w->mg, p, x, st);
        if (rc) return rc;
    }
    if (pc32) {
        FE_CHECK_HIP((launch_cast<double, float>(x, w->x32, p->ndof, st)));
        FE_CHECK_HIP((launch_blockdiag<float>(p->geo, w->x32, gamma, s_elem, p->nmask, w->D32,
                                              reinterpret_cast<float *>(p->slots25), st)));
        FE_CHECK_HIP(launch_invert_blocks32(w->D32, p->nn, st));
    } else {
        FE_CHECK_HIP(launch_blockdiag(p->geo, x, gamma, s_elem, p->nmask, w->D, p->slots25, st));
        FE_CHECK_HIP(launch_invert_blocks(w->D, nullptr, p->nn, st));
    }
    if (pc == FE_PC_MULTIGRID) {
        rc = mg_setup_finish(w->mg, p, w->D, pc32 ? w->D32 : nullptr, pc32 ? w->x32 : nullptr, st);
        if (rc) return rc;
    }
    LinSys L;
    L.z32 = pc32;
    L.op32 = false;
    L.prec = [&](const double *v, void *z) -> hipError_t {
        if (pc == FE_PC_MULTIGRID) {
            const int r = pc32 ? mg_apply32(w->mg, v, (float *)z, true, st)
                               : mg_apply64(w->mg, v, (double *)z, true, st);
            return r == FE_OK ? hipSuccess : hipErrorUnknown;
        }
        if (pc32)
            return launch_block_apply<float, double, float>(w->D32, v, (float *)z, p->nn, true,
                                                            nullptr, st);
        return launch_block_apply<double, double, double>(w->D, v, (double *)z, p->nn, true,
                                                          nullptr, st);
    };
    L.op_z = [&](const void *z, double *out) -> hipError_t {
        if (pc32)  // FP32 z_j, widened as the FP64 operator stages it
            return launch_elem_dir32(OP_JTV, p->geo, x, (const float *)z, gamma, s_elem,
                                     p->nmask, out, p->slots, st);
        return launch_elem<double, double>(OP_JTV, p->geo, x, (const double *)z, gamma, s_elem,
                                           p->nmask, out, p->slots, st);
    };
    L.op64 = [&](const double *v, double *out) -> hipError_t {
        return launch_elem<double, double>(OP_JTV, p->geo, x, v, gamma, s_elem, p->nmask, out,
                                           p->slots, st);
    };
    LinStats ls;
    rc = fgmres(p, L, rhs, lambda, opts.rtol_lin, opts.restart, opts.max_lin, 0, st, &ls,
                opts.verbose);
    if (rc) return rc;
    FE_CHECK_HIP(hipStreamSynchronize(st));
    rep.lin_its_total = ls.its;
    rep.lin_its[0] = ls.its;
    rep.status = ls.converged ? FE_OK : FE_NOT_CONVERGED;
    rep.res_final = ls.res_true;
    rep.t_jv_s = ls.t_jv;
    rep.t_prec_s = ls.t_prec;
    rep.t_orth_s = ls.t_orth;
    rep.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rep.precond = pc;
    rep.mg_levels = pc == FE_PC_MULTIGRID ? (int)w->mg->lev.size() : 0;
    fill_report(report, rep);
    if (!ls.converged) set_error("fe_adjoint_solve: FGMRES not converged");
    return rep.status;
}

}  // extern "C"
