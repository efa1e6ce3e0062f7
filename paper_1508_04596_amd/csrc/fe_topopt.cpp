// C-ABI of the optimisation loop (Sec. "Optimisation problem" and Sec.
// "Continuation scheme"): the PDE density filter, MMA, and the design loop that
// chains filter -> state solve -> thermal compliance -> adjoint -> design
// sensitivities -> filter transpose -> MMA, with the five-step continuation
// on (q_f, q_alpha, alpha_max) and warm-started state solves.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fe_topopt.h"

using namespace fe;

struct fe_filter {
    Filter f;
    fe_grid grid;
};

struct fe_mma {
    MmaState m;
};

struct fe_topopt {
    fe_problem *p = nullptr;
    const uint8_t *design = nullptr;
    const double *gamma_fixed = nullptr, *s = nullptr;
    fe_topopt_opts o;
    Filter filt;
    MmaState mma;
    int64_t ne = 0, nd = 0;
    int64_t *idx = nullptr;               // design element indices
    double *gin = nullptr, *gt = nullptr;  // blended and filtered design fields
    double *lam = nullptr, *dfdx = nullptr;
    double *ge = nullptr, *tmp = nullptr;  // element work
    double *df0 = nullptr, *df1 = nullptr, *rc = nullptr, *rc_old = nullptr;  // compact
    double *partial = nullptr;
    std::vector<double> hpart;
    double f_ref = 0.0;
    int iter = 0;
};

static int filter_apply_impl(Filter *f, const double *in, double *out, bool transpose,
                             double h, hipStream_t st)
{
    const double load = h * h * h / 8.0;
    FE_CHECK_HIP(filter_load(f, in, transpose ? 0.125 : load, st));
    int rc = filter_solve(f, st, 1e-12, 5000);
    if (rc != FE_OK) {
        set_error(rc == FE_ENAN ? "filter: non-finite field" : "filter: CG not converged");
        return rc;
    }
    FE_CHECK_HIP(filter_unload(f, transpose ? load : 0.125, out, st));
    return FE_OK;
}

extern "C" {

// ---- filter ---------------------------------------------------------------------------

int fe_filter_create(const fe_grid *grid, double radius, fe_filter **out)
{
    if (!grid || !out || grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || !(grid->h > 0) ||
        !(radius >= 0) || !std::isfinite(radius)) {
        set_error("fe_filter_create: bad grid or radius");
        return FE_EINVAL;
    }
    auto *F = new (std::nothrow) fe_filter();
    if (!F) return FE_ENOMEM;
    F->grid = *grid;
    hipError_t e = filter_alloc(&F->f, *grid, radius);
    if (e != hipSuccess) {
        filter_free(&F->f);
        delete F;
        return hip_fail(e, "fe_filter_create");
    }
    *out = F;
    return FE_OK;
}

int fe_filter_apply(fe_filter *F, const double *in, double *out, hipStream_t st)
{
    if (!F || !in || !out) {
        set_error("fe_filter_apply: NULL argument");
        return FE_EINVAL;
    }
    return filter_apply_impl(&F->f, in, out, false, F->grid.h, st);
}

int fe_filter_apply_transpose(fe_filter *F, const double *in, double *out, hipStream_t st)
{
    if (!F || !in || !out) {
        set_error("fe_filter_apply_transpose: NULL argument");
        return FE_EINVAL;
    }
    return filter_apply_impl(&F->f, in, out, true, F->grid.h, st);
}

int fe_filter_iterations(const fe_filter *F) { return F ? F->f.last_its : -1; }

int fe_filter_destroy(fe_filter *F)
{
    if (!F) return FE_OK;
    filter_free(&F->f);
    delete F;
    return FE_OK;
}

// ---- MMA --------------------------------------------------------------------------------

int fe_mma_create(int64_t n, double xmin, double xmax, double move, fe_mma **out)
{
    if (!out || n < 1 || !(xmax > xmin) || !(move > 0)) {
        set_error("fe_mma_create: need n >= 1, xmax > xmin, move > 0");
        return FE_EINVAL;
    }
    auto *M = new (std::nothrow) fe_mma();
    if (!M) return FE_ENOMEM;
    M->m.n = n;
    M->m.xmin = xmin;
    M->m.xmax = xmax;
    M->m.move = move;
    hipError_t e = mma_alloc(&M->m);
    if (e != hipSuccess) {
        mma_free(&M->m);
        delete M;
        return hip_fail(e, "fe_mma_create");
    }
    *out = M;
    return FE_OK;
}

int fe_mma_update(fe_mma *M, double *x, const double *df0, double f1, const double *df1,
                  double *lambda_out, hipStream_t st)
{
    if (!M || !x || !df0 || !df1) {
        set_error("fe_mma_update: NULL argument");
        return FE_EINVAL;
    }
    return mma_update(&M->m, x, df0, f1, df1, lambda_out, st);
}

int fe_mma_destroy(fe_mma *M)
{
    if (!M) return FE_OK;
    mma_free(&M->m);
    delete M;
    return FE_OK;
}

// ---- design loop ------------------------------------------------------------------------

void fe_topopt_opts_default(fe_topopt_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    const double qf[5] = {0.881, 8.81, 88.1, 881.0, 881.0};
    const double qa[5] = {8.0, 8.0, 8.0, 98.0, 998.0};
    const double am[5] = {1e5, 1e5, 1e5, 1e6, 1e7};
    o->n_steps = 5;
    for (int k = 0; k < 5; ++k) {
        o->iters_per_step[k] = 100;
        o->q_f[k] = qf[k];
        o->q_alpha[k] = qa[k];
        o->alpha_max[k] = am[k];
    }
    o->vf = 0.05;
    o->filter_radius = 2.5;
    o->move = 0.2;
    fe_solve_opts_default(&o->state);
    o->state.rtol_newton = 1e-4;
    o->state.ramp_steps = 4;
    fe_solve_opts_default(&o->adjoint);
    o->adjoint.rtol_lin = 1e-6;
}

int fe_topopt_destroy(fe_topopt *T)
{
    if (!T) return FE_OK;
    filter_free(&T->filt);
    mma_free(&T->mma);
    for (void *q : {(void *)T->idx, (void *)T->gin, (void *)T->gt, (void *)T->lam,
                    (void *)T->dfdx, (void *)T->ge, (void *)T->tmp, (void *)T->df0,
                    (void *)T->df1, (void *)T->rc, (void *)T->rc_old, (void *)T->partial})
        if (q) (void)hipFree(q);
    delete T;
    return FE_OK;
}

int fe_topopt_create(fe_problem *p, const uint8_t *design_mask, const double *gamma_fixed,
                     const double *s_elem, const fe_topopt_opts *opts, fe_topopt **out)
{
    if (!p || !design_mask || !gamma_fixed || !s_elem || !out) {
        set_error("fe_topopt_create: NULL argument");
        return FE_EINVAL;
    }
    auto *T = new (std::nothrow) fe_topopt();
    if (!T) return FE_ENOMEM;
    T->p = p;
    T->design = design_mask;
    T->gamma_fixed = gamma_fixed;
    T->s = s_elem;
    fe_topopt_opts_default(&T->o);
    if (opts) T->o = *opts;
    if (T->o.n_steps < 1 || T->o.n_steps > 5 || !(T->o.vf > 0 && T->o.vf < 1) ||
        !(T->o.filter_radius >= 0) || !(T->o.move > 0)) {
        delete T;
        set_error("fe_topopt_create: bad options (n_steps 1..5, 0 < vf < 1, radius >= 0, move > 0)");
        return FE_EINVAL;
    }
    T->ne = p->ne;
    // design element indices (host side once)
    std::vector<uint8_t> hm(T->ne);
    hipError_t e = hipMemcpy(hm.data(), design_mask, T->ne, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        delete T;
        return hip_fail(e, "fe_topopt_create: design mask");
    }
    std::vector<int64_t> hidx;
    for (int64_t i = 0; i < T->ne; ++i)
        if (hm[i]) hidx.push_back(i);
    T->nd = (int64_t)hidx.size();
    if (T->nd == 0) {
        delete T;
        set_error("fe_topopt_create: empty design domain");
        return FE_EINVAL;
    }
    const size_t be = sizeof(double) * T->ne, bd = sizeof(double) * T->nd,
                 bx = sizeof(double) * p->ndof;
    e = filter_alloc(&T->filt, p->grid, T->o.filter_radius * p->grid.h);
    T->mma.n = T->nd;
    T->mma.move = T->o.move;
    if (e == hipSuccess) e = mma_alloc(&T->mma);
    if (e == hipSuccess) e = hipMalloc(&T->idx, sizeof(int64_t) * T->nd);
    if (e == hipSuccess) e = hipMalloc(&T->gin, be);
    if (e == hipSuccess) e = hipMalloc(&T->gt, be);
    if (e == hipSuccess) e = hipMalloc(&T->ge, be);
    if (e == hipSuccess) e = hipMalloc(&T->tmp, be);
    if (e == hipSuccess) e = hipMalloc(&T->lam, bx);
    if (e == hipSuccess) e = hipMalloc(&T->dfdx, bx);
    if (e == hipSuccess) e = hipMalloc(&T->df0, bd);
    if (e == hipSuccess) e = hipMalloc(&T->df1, bd);
    if (e == hipSuccess) e = hipMalloc(&T->rc, bd);
    if (e == hipSuccess) e = hipMalloc(&T->rc_old, bd);
    if (e == hipSuccess) e = hipMalloc(&T->partial, sizeof(double) * 2 * RED_BLOCKS);
    if (e == hipSuccess)
        e = hipMemcpy(T->idx, hidx.data(), sizeof(int64_t) * T->nd, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        fe_topopt_destroy(T);
        return hip_fail(e, "fe_topopt_create");
    }
    T->hpart.resize(2 * RED_BLOCKS);
    *out = T;
    return FE_OK;
}

// objective, volume constraint and their design gradients at rho
static int evaluate(fe_topopt *T, const double *rho, double *x, double *f, double *g,
                    double *dfdrho, double *dgdrho, fe_topopt_record *rec, hipStream_t st)
{
    fe_problem *p = T->p;
    const double h = p->grid.h;
    auto t0 = std::chrono::steady_clock::now();
    // physical design: design elements filtered, the rest fixed
    FE_CHECK_HIP(launch_blend(T->ne, T->design, rho, T->gamma_fixed, T->gin, st));
    int rc = filter_apply_impl(&T->filt, T->gin, T->gt, false, h, st);
    if (rc) return rc;
    FE_CHECK_HIP(launch_blend(T->ne, T->design, T->gt, T->gamma_fixed, T->gt, st));
    // state (warm start from x)
    fe_solve_report rs;
    rc = newton_solve(p, T->gt, T->s, x, &T->o.state, &rs, st);
    if (rc != FE_OK) return rc;
    auto t1 = std::chrono::steady_clock::now();
    // objective and adjoint
    double fv = 0.0;
    rc = fe_compliance(p, x, T->s, &fv, T->dfdx, st);
    if (rc) return rc;
    fe_solve_report ra;
    rc = fe_adjoint_solve(p, x, T->gt, T->s, T->dfdx, T->lam, &T->o.adjoint, &ra, st);
    if (rc != FE_OK) return rc;
    auto t2 = std::chrono::steady_clock::now();
    // df/dgamma~ = -lambda^T dR/dgamma on the design; through the filter transpose
    rc = fe_dR_dgamma(p, x, T->gt, T->s, T->lam, T->ge, st);
    if (rc) return rc;
    if (dfdrho) {
        FE_CHECK_HIP(launch_masked_scale(T->ne, T->design, T->ge, -1.0, T->tmp, st));
        rc = filter_apply_impl(&T->filt, T->tmp, dfdrho, true, h, st);
        if (rc) return rc;
        FE_CHECK_HIP(launch_masked_scale(T->ne, T->design, dfdrho, 1.0, dfdrho, st));
    }
    // volume: g = mean over the design of (1 - gamma~) - vf
    FE_CHECK_HIP(launch_vol_change(T->ne, T->design, T->gt, 0, nullptr, nullptr, T->partial, st));
    FE_CHECK_HIP(hipMemcpyAsync(T->hpart.data(), T->partial, sizeof(double) * RED_BLOCKS,
                                hipMemcpyDeviceToHost, st));
    FE_CHECK_HIP(hipStreamSynchronize(st));
    double vs = 0.0;
    for (int b = 0; b < RED_BLOCKS; ++b) vs += T->hpart[b];
    const double gv = vs / (double)T->nd - T->o.vf;
    if (dgdrho) {
        FE_CHECK_HIP(launch_masked_scale(T->ne, T->design, nullptr, -1.0 / (double)T->nd, T->tmp, st));
        rc = filter_apply_impl(&T->filt, T->tmp, dgdrho, true, h, st);
        if (rc) return rc;
        FE_CHECK_HIP(launch_masked_scale(T->ne, T->design, dgdrho, 1.0, dgdrho, st));
    }
    FE_CHECK_HIP(hipStreamSynchronize(st));
    auto t3 = std::chrono::steady_clock::now();
    *f = fv;
    *g = gv;
    if (rec) {
        rec->f = fv;
        rec->g = gv;
        rec->newton_its = rs.newton_its;
        rec->lin_its = rs.lin_its_total;
        rec->adj_its = ra.lin_its_total;
        rec->ramp_stages = rs.ramp_stages;
        rec->t_state_s = std::chrono::duration<double>(t1 - t0).count();
        rec->t_adjoint_s = std::chrono::duration<double>(t2 - t1).count();
        rec->t_total_s = std::chrono::duration<double>(t3 - t0).count();
    }
    return FE_OK;
}

int fe_topopt_evaluate(fe_topopt *T, const double *rho, double *x, double *f, double *g,
                       double *dfdrho, double *dgdrho, fe_topopt_record *rec, hipStream_t st)
{
    if (!T || !rho || !x || !f || !g) {
        set_error("fe_topopt_evaluate: NULL argument");
        return FE_EINVAL;
    }
    if (rec) std::memset(rec, 0, sizeof(*rec));
    return evaluate(T, rho, x, f, g, dfdrho, dgdrho, rec, st);
}

int fe_topopt_step(fe_topopt *T, double *rho, double *x, fe_topopt_record *rec, hipStream_t st)
{
    if (!T || !rho || !x) {
        set_error("fe_topopt_step: NULL argument");
        return FE_EINVAL;
    }
    fe_topopt_record r;
    std::memset(&r, 0, sizeof(r));
    auto t0 = std::chrono::steady_clock::now();
    double f = 0.0, g = 0.0;
    int rc = evaluate(T, rho, x, &f, &g, T->ge, T->tmp, &r, st);
    if (rc) return rc;
    if (T->iter == 0) T->f_ref = f;
    const double fs = T->f_ref != 0.0 ? 1.0 / T->f_ref : 1.0;
    // compact design vectors; objective scaled by its first value
    FE_CHECK_HIP(launch_gather(T->nd, T->idx, T->ge, T->df0, st));
    FE_CHECK_HIP(launch_axpby(T->nd, fs, T->df0, 0.0, T->df0, st));
    FE_CHECK_HIP(launch_gather(T->nd, T->idx, T->tmp, T->df1, st));
    FE_CHECK_HIP(launch_gather(T->nd, T->idx, rho, T->rc, st));
    FE_CHECK_HIP(hipMemcpyAsync(T->rc_old, T->rc, sizeof(double) * T->nd, hipMemcpyDeviceToDevice, st));
    double lam = 0.0;
    rc = mma_update(&T->mma, T->rc, T->df0, g, T->df1, &lam, st);
    if (rc) return rc;
    FE_CHECK_HIP(launch_scatter(T->nd, T->idx, T->rc, rho, st));
    // largest design change
    FE_CHECK_HIP(launch_vol_change(0, T->design, T->gt, T->nd, T->rc, T->rc_old, T->partial, st));
    FE_CHECK_HIP(hipMemcpyAsync(T->hpart.data(), T->partial, sizeof(double) * 2 * RED_BLOCKS,
                                hipMemcpyDeviceToHost, st));
    FE_CHECK_HIP(hipStreamSynchronize(st));
    double ch = 0.0;
    for (int b = 0; b < RED_BLOCKS; ++b) ch = std::max(ch, T->hpart[RED_BLOCKS + b]);
    r.iter = T->iter++;
    r.f_scaled = f * fs;
    r.change = ch;
    r.lambda_mma = lam;
    r.t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rec) *rec = r;
    return FE_OK;
}

int fe_topopt_run(fe_topopt *T, double *rho, double *x, fe_topopt_record *hist, int cap,
                  int *n_done, hipStream_t st)
{
    if (!T || !rho || !x) {
        set_error("fe_topopt_run: NULL argument");
        return FE_EINVAL;
    }
    int done = 0;
    for (int k = 0; k < T->o.n_steps; ++k) {
        fe_phys ph = T->p->phys;
        ph.qf = T->o.q_f[k];
        ph.q_alpha = T->o.q_alpha[k];
        ph.alpha_max = T->o.alpha_max[k];
        int rc = fe_problem_set_phys(T->p, &ph);
        if (rc) return rc;
        for (int it = 0; it < T->o.iters_per_step[k]; ++it) {
            fe_topopt_record r;
            rc = fe_topopt_step(T, rho, x, &r, st);
            if (rc) {
                if (n_done) *n_done = done;
                return rc;
            }
            r.step = k;
            if (hist && done < cap) hist[done] = r;
            ++done;
        }
    }
    if (n_done) *n_done = done;
    return FE_OK;
}

}  // extern "C"
