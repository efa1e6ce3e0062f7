// C-ABI entry points: problem handle, operators, objective.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "fe_internal.h"
#include "fe_mg.h"

namespace fe {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char *what)
{
    set_error(std::string("HIP error ") + hipGetErrorString(e) + " in " + what);
    return e == hipErrorOutOfMemory ? FE_ENOMEM : FE_EHIP;
}

Geo make_geo(const fe_grid &g, const fe_phys &ph)
{
    Geo o;
    o.nx = g.nx;
    o.ny = g.ny;
    o.nz = g.nz;
    o.ntx = (g.nx + TX - 1) / TX;
    o.nty = (g.ny + TY - 1) / TY;
    o.ntz = (g.nz + TZ - 1) / TZ;
    o.h = g.h;
    o.Pr = ph.Pr;
    o.B = ph.Gr * ph.Pr * ph.Pr;
    for (int d = 0; d < 3; ++d) o.eg[d] = ph.eg[d];
    o.Ck = ph.Ck;
    o.qf = ph.qf;
    o.amax = ph.alpha_max;
    o.qa = ph.q_alpha;
    const double h = g.h;
    o.W = 0.125 * h * h * h;
    o.gs = 2.0 * 1.7320508075688772935 / h;
    o.igs = h / (2.0 * 1.7320508075688772935);
    o.inv16h2 = 1.0 / (16.0 * h * h);
    o.cvisc = 16.0 * ph.Pr * ph.Pr / (h * h * h * h);
    o.c16h4 = 16.0 / (h * h * h * h);
    return o;
}

static int check_grid(const fe_grid *g)
{
    if (!g) {
        set_error("grid is NULL");
        return FE_EINVAL;
    }
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->h > 0.0) || !std::isfinite(g->h)) {
        set_error("grid sizes must be >= 1 and h > 0");
        return FE_EINVAL;
    }
    const int64_t nn = (int64_t)(g->nx + 1) * (g->ny + 1) * (g->nz + 1);
    if (nn > (int64_t)1 << 31) {
        set_error("grid too large: node count exceeds 2^31");
        return FE_EINVAL;
    }
    return FE_OK;
}

static int check_phys(const fe_phys *ph)
{
    if (!ph) {
        set_error("phys is NULL");
        return FE_EINVAL;
    }
    if (!(ph->Ck > 0.0) || !std::isfinite(ph->Pr) || !std::isfinite(ph->Gr) ||
        !std::isfinite(ph->alpha_max)) {
        set_error("phys: Ck must be > 0 and Pr, Gr, alpha_max finite");
        return FE_EINVAL;
    }
    return FE_OK;
}

namespace {
struct HipAllocator final : Allocator {
    hipError_t dev_alloc(void **p, size_t n) override { return hipMalloc(p, n); }
    void dev_free(void *p) override { (void)hipFree(p); }
    hipError_t host_alloc(void **p, size_t n) override { return hipHostMalloc(p, n); }
    void host_free(void *p) override { (void)hipHostFree(p); }
};
}  // namespace

Allocator *default_allocator()
{
    static HipAllocator a;
    return &a;
}

int problem_create_ex(const fe_grid *grid, const fe_phys *phys, const uint8_t *dof_mask,
                      MaskKind kind, Allocator *alloc, hipStream_t stream, fe_problem **out)
{
    if (!out) {
        set_error("out is NULL");
        return FE_EINVAL;
    }
    *out = nullptr;
    int rc = check_grid(grid);
    if (rc) return rc;
    rc = check_phys(phys);
    if (rc) return rc;
    fe_problem *p = new (std::nothrow) fe_problem();
    if (!p) return FE_ENOMEM;
    p->alloc = alloc ? alloc : default_allocator();
    p->grid = *grid;
    p->phys = *phys;
    p->geo = make_geo(*grid, *phys);
    p->nn = n_nodes(p->geo);
    p->ne = n_elem(p->geo);
    p->ndof = NF * p->nn;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDevice");
    }
    const size_t slot_bytes = (size_t)n_tiles(p->geo) * BOXN * NF * sizeof(double);
    if ((e = dalloc(p, &p->nmask, p->nn)) != hipSuccess ||
        (e = dalloc(p, &p->dof_mask, p->ndof)) != hipSuccess ||
        (e = dalloc(p, &p->slots, slot_bytes)) != hipSuccess ||
        (e = dalloc(p, &p->partial, sizeof(double) * PARTIAL_COLS * RED_BLOCKS)) != hipSuccess ||
        (e = dalloc(p, &p->scal, sizeof(double) * 256)) != hipSuccess) {
        fe_problem_destroy(p);
        return hip_fail(e, "device allocation (problem)");
    }
    if (kind == MASK_WALLS_PIN) {
        e = launch_wall_mask(grid->nx, grid->ny, grid->nz, p->nmask, p->dof_mask, stream);
    } else {
        if (dof_mask)
            e = hipMemcpyAsync(p->dof_mask, dof_mask, p->ndof, hipMemcpyDeviceToDevice, stream);
        else
            e = hipMemsetAsync(p->dof_mask, 0, p->ndof, stream);
        if (e == hipSuccess) e = launch_node_mask(p->dof_mask, p->nmask, p->nn, stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        fe_problem_destroy(p);
        return hip_fail(e, "fe_problem_create mask setup");
    }
    *out = p;
    return FE_OK;
}

}  // namespace fe

using namespace fe;

extern "C" {

const char *fe_last_error(void) { return g_last_error.c_str(); }
const char *fe_version(void) { return "fe-hip 1.0 (gfx950)"; }

int fe_problem_create(const fe_grid *grid, const fe_phys *phys, const uint8_t *dof_mask,
                      fe_problem **out)
{
    return problem_create_ex(grid, phys, dof_mask, MASK_GIVEN, nullptr, 0, out);
}

void fe_free_solver_ws(fe_problem *p);  // fe_solver.cpp

int fe_problem_destroy(fe_problem *p)
{
    if (!p) return FE_OK;
    for (hipEvent_t e : p->timer_ev) (void)hipEventDestroy(e);
    fe_free_solver_ws(p);
    dfree(p, p->nmask);
    dfree(p, p->dof_mask);
    dfree(p, p->slots);
    dfree(p, p->slots25);
    dfree(p, p->partial);
    dfree(p, p->scal);
    delete p;
    return FE_OK;
}

int fe_problem_set_phys(fe_problem *p, const fe_phys *phys)
{
    if (!p) {
        set_error("problem is NULL");
        return FE_EINVAL;
    }
    int rc = check_phys(phys);
    if (rc) return rc;
    p->phys = *phys;
    p->geo = make_geo(p->grid, *phys);
    return FE_OK;
}

int64_t fe_problem_ndof(const fe_problem *p) { return p ? p->ndof : -1; }

int fe_residual(fe_problem *p, const double *x, const double *gamma, const double *s_elem,
                double *r, hipStream_t stream)
{
    if (!p || !x || !gamma || !s_elem || !r) {
        set_error("fe_residual: NULL argument");
        return FE_EINVAL;
    }
    FE_CHECK_HIP((launch_elem<double, double>(OP_RES, p->geo, x, (const double *)nullptr, gamma,
                                              s_elem, p->nmask, r, p->slots, stream)));
    return FE_OK;
}

int fe_jvp(fe_problem *p, fe_prec prec, const void *x, const double *gamma, const double *s_elem,
           const void *v, void *jv, hipStream_t stream)
{
    if (!p || !x || !gamma || !s_elem || !v || !jv) {
        set_error("fe_jvp: NULL argument");
        return FE_EINVAL;
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (p->timer_on) {
        while (p->timer_ev.size() < 2 * (p->timer_n + 1)) {
            hipEvent_t e;
            FE_CHECK_HIP(hipEventCreate(&e));
            p->timer_ev.push_back(e);
        }
        ev0 = p->timer_ev[2 * p->timer_n];
        ev1 = p->timer_ev[2 * p->timer_n + 1];
    }
    if (prec == FE_FP64) {
        FE_CHECK_HIP((launch_elem<double, double>(OP_JV, p->geo, (const double *)x,
                                                  (const double *)v, gamma, s_elem, p->nmask,
                                                  (double *)jv, p->slots, stream, ev0, ev1)));
    } else if (prec == FE_FP32) {
        FE_CHECK_HIP((launch_elem<float, float>(OP_JV, p->geo, (const float *)x, (const float *)v,
                                                gamma, s_elem, p->nmask, (float *)jv,
                                                (float *)p->slots, stream, ev0, ev1)));
    } else {
        set_error("fe_jvp: unknown precision");
        return FE_EINVAL;
    }
    if (p->timer_on) ++p->timer_n;
    return FE_OK;
}

int fe_kernel_timer(fe_problem *p, int enable)
{
    if (!p) {
        set_error("fe_kernel_timer: NULL problem");
        return FE_EINVAL;
    }
    p->timer_on = enable != 0;
    p->timer_n = 0;
    return FE_OK;
}

int fe_kernel_timer_read(fe_problem *p, double *elem_ms, int64_t *launches)
{
    if (!p || !elem_ms || !launches) {
        set_error("fe_kernel_timer_read: NULL argument");
        return FE_EINVAL;
    }
    double total = 0.0;
    for (size_t i = 0; i < p->timer_n; ++i) {
        float ms = 0.f;
        FE_CHECK_HIP(hipEventSynchronize(p->timer_ev[2 * i + 1]));
        FE_CHECK_HIP(hipEventElapsedTime(&ms, p->timer_ev[2 * i], p->timer_ev[2 * i + 1]));
        total += ms;
    }
    *elem_ms = total;
    *launches = (int64_t)p->timer_n;
    p->timer_n = 0;
    return FE_OK;
}

int fe_adjoint_jtvp(fe_problem *p, fe_prec prec, const void *x, const double *gamma,
                    const double *s_elem, const void *w, void *jtw, hipStream_t stream)
{
    if (!p || !x || !gamma || !s_elem || !w || !jtw) {
        set_error("fe_adjoint_jtvp: NULL argument");
        return FE_EINVAL;
    }
    if (prec == FE_FP64) {
        FE_CHECK_HIP((launch_elem<double, double>(OP_JTV, p->geo, (const double *)x,
                                                  (const double *)w, gamma, s_elem, p->nmask,
                                                  (double *)jtw, p->slots, stream)));
    } else if (prec == FE_FP32) {
        FE_CHECK_HIP((launch_elem<float, float>(OP_JTV, p->geo, (const float *)x, (const float *)w,
                                                gamma, s_elem, p->nmask, (float *)jtw,
                                                (float *)p->slots, stream)));
    } else {
        set_error("fe_adjoint_jtvp: unknown precision");
        return FE_EINVAL;
    }
    return FE_OK;
}

int fe_dR_dgamma(fe_problem *p, const double *x, const double *gamma, const double *s_elem,
                 const double *lambda, double *g_elem, hipStream_t stream)
{
    if (!p || !x || !gamma || !s_elem || !lambda || !g_elem) {
        set_error("fe_dR_dgamma: NULL argument");
        return FE_EINVAL;
    }
    FE_CHECK_HIP(launch_dRdgamma(p->geo, x, lambda, gamma, s_elem, p->nmask, g_elem, stream));
    return FE_OK;
}

int fe_block_diagonal(fe_problem *p, const double *x, const double *gamma, const double *s_elem,
                      double *D, hipStream_t stream)
{
    if (!p || !x || !gamma || !s_elem || !D) {
        set_error("fe_block_diagonal: NULL argument");
        return FE_EINVAL;
    }
    if (!p->slots25) {
        const size_t b = (size_t)n_tiles(p->geo) * BOXN * 25 * sizeof(double);
        FE_CHECK_HIP(dalloc(p, &p->slots25, b));
    }
    FE_CHECK_HIP((launch_blockdiag<double>(p->geo, x, gamma, s_elem, p->nmask, D, p->slots25, stream)));
    return FE_OK;
}

int fe_block_diagonal_fp32(fe_problem *p, const float *x, const double *gamma,
                           const double *s_elem, float *D, hipStream_t stream)
{
    if (!p || !x || !gamma || !s_elem || !D) {
        set_error("fe_block_diagonal_fp32: NULL argument");
        return FE_EINVAL;
    }
    if (!p->slots25) {
        const size_t b = (size_t)n_tiles(p->geo) * BOXN * 25 * sizeof(double);
        FE_CHECK_HIP(dalloc(p, &p->slots25, b));
    }
    FE_CHECK_HIP((launch_blockdiag<float>(p->geo, x, gamma, s_elem, p->nmask, D,
                                          reinterpret_cast<float *>(p->slots25), stream)));
    return FE_OK;
}

int fe_jacobian_dense(fe_problem *p, const double *x, const double *gamma, const double *s_elem,
                      double *J_host, hipStream_t stream)
{
    if (!p || !x || !gamma || !s_elem || !J_host) {
        set_error("fe_jacobian_dense: NULL argument");
        return FE_EINVAL;
    }
    if (p->ndof > FE_DENSE_MAX_DOF) {
        set_error("fe_jacobian_dense: more than FE_DENSE_MAX_DOF unknowns");
        return FE_EINVAL;
    }
    double *Je = nullptr, *probe = nullptr;
    double *h = nullptr;
    hipError_t e = dalloc(p, &Je, sizeof(double) * 1600 * p->ne);
    if (e == hipSuccess) e = dalloc(p, &probe, sizeof(double) * 135 * p->ndof);
    if (e == hipSuccess) e = halloc(p, &h, sizeof(double) * 135 * p->ndof);
    if (e == hipSuccess)
        e = launch_probe_products(p->geo, x, gamma, s_elem, p->nmask, Je, probe, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h, probe, sizeof(double) * 135 * p->ndof, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess) assemble_from_probes(p->grid, h, J_host);
    dfree(p, Je);
    dfree(p, probe);
    hfree(p, h);
    if (e != hipSuccess) return hip_fail(e, "fe_jacobian_dense");
    return FE_OK;
}

int fe_compliance(fe_problem *p, const double *x, const double *s_elem, double *f_host,
                  double *dfdx, hipStream_t stream)
{
    if (!p || !x || !s_elem) {
        set_error("fe_compliance: NULL argument");
        return FE_EINVAL;
    }
    FE_CHECK_HIP(launch_compliance(p->geo, x, s_elem, p->nmask, dfdx, p->partial, stream));
    if (f_host) {
        FE_CHECK_HIP(launch_reduce(p->partial, 1, p->scal, nullptr, false, stream));
        FE_CHECK_HIP(hipMemcpyAsync(f_host, p->scal, sizeof(double), hipMemcpyDeviceToHost, stream));
        FE_CHECK_HIP(hipStreamSynchronize(stream));
    }
    return FE_OK;
}

double fe_line_search_lambda(double phi0, double phi_half, double phi1, double lambda_min)
{
    // quadratic q(l) = phi0 + c1 l + c2 l^2 through l = 0, 1/2, 1
    const double c2 = 2.0 * (phi1 - 2.0 * phi_half + phi0);
    const double c1 = phi1 - phi0 - c2;
    if (c2 > 0.0) {
        double l = -c1 / (2.0 * c2);
        if (l > 1.0) l = 1.0;
        if (l < lambda_min) l = lambda_min;
        return l;
    }
    return (phi_half < phi1) ? 0.5 : 1.0;
}

}  // extern "C"
