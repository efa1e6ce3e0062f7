// Method of moving asymptotes for one constraint (Sec. "Optimisation
// problem": the design problem is solved with MMA), on the device.
//
// Per variable: moving asymptotes, subproblem bounds and the coefficients of
// the convex separable approximations of the objective and of the constraint
// (published MMA safeguards: asymptote factors 0.5 / 1.2 / 0.7, asymptote
// distance within [0.01, 10] of the box, bounds 10 % inside the asymptotes,
// move limit, gradient split 1.001 / 0.001 plus 1e-5 regularisation).  The dual
// of the subproblem is one-dimensional: for a multiplier lam each variable has
// a closed-form minimiser, and the constraint approximation at that point is
// a deterministic block-partial sum; the host brackets and bisects lam.
#include "fe_topopt.h"

namespace fe {
namespace {

struct MmaPar {
    double xmin, xmax, move;
    int first;  // first two iterations: initial asymptotes
};

__device__ __forceinline__ double xlam(double lam, double p0, double q0, double p1, double q1,
                                       double low, double upp, double al, double be)
{
    const double sP = sqrt(p0 + lam * p1), sQ = sqrt(q0 + lam * q1);
    const double xs = (sP * low + sQ * upp) / (sP + sQ);
    return fmin(fmax(xs, al), be);
}

template <int NV>
__device__ __forceinline__ void mma_partials(double v[NV], double *partial)
{
    __shared__ double red[NV][RED_THREADS / 64];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double s = v[j];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
        if ((threadIdx.x & 63) == 0) red[j][threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < RED_THREADS / 64; ++w) s += red[threadIdx.x][w];
        partial[threadIdx.x * RED_BLOCKS + blockIdx.x] = s;
    }
}

// asymptotes, bounds, approximation coefficients; partial sums of the
// constraint approximation's variable part at x (for r1)
__global__ __launch_bounds__(RED_THREADS) void k_mma_prep(
    MmaPar P, int64_t n, const double *__restrict__ x, const double *__restrict__ df0,
    const double *__restrict__ df1, const double *__restrict__ xold1,
    const double *__restrict__ xold2, double *__restrict__ low, double *__restrict__ upp,
    double *__restrict__ al, double *__restrict__ be, double *__restrict__ c, double *partial)
{
    const double d = P.xmax - P.xmin, reg = 1e-5 / d;
    double v[1] = {0.0};
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double xj = x[j];
        double lo, up;
        if (P.first) {
            lo = xj - 0.5 * d;
            up = xj + 0.5 * d;
        } else {
            const double zz = (xj - xold1[j]) * (xold1[j] - xold2[j]);
            const double s = zz > 0.0 ? 1.2 : (zz < 0.0 ? 0.7 : 1.0);
            lo = xj - s * (xold1[j] - low[j]);
            up = xj + s * (upp[j] - xold1[j]);
            lo = fmin(fmax(lo, xj - 10.0 * d), xj - 0.01 * d);
            up = fmax(fmin(up, xj + 10.0 * d), xj + 0.01 * d);
        }
        low[j] = lo;
        upp[j] = up;
        al[j] = fmax(fmax(P.xmin, lo + 0.1 * (xj - lo)), xj - P.move * d);
        be[j] = fmin(fmin(P.xmax, up - 0.1 * (up - xj)), xj + P.move * d);
        const double ux2 = (up - xj) * (up - xj), xl2 = (xj - lo) * (xj - lo);
        const double a0 = fmax(df0[j], 0.0), b0 = fmax(-df0[j], 0.0);
        const double a1 = fmax(df1[j], 0.0), b1 = fmax(-df1[j], 0.0);
        const double p0 = ux2 * (1.001 * a0 + 0.001 * b0 + reg), q0 = xl2 * (0.001 * a0 + 1.001 * b0 + reg);
        const double p1 = ux2 * (1.001 * a1 + 0.001 * b1 + reg), q1 = xl2 * (0.001 * a1 + 1.001 * b1 + reg);
        c[4 * j + 0] = p0;
        c[4 * j + 1] = q0;
        c[4 * j + 2] = p1;
        c[4 * j + 3] = q1;
        v[0] += p1 / (up - xj) + q1 / (xj - lo);
    }
    mma_partials<1>(v, partial);
}

// partial sums of the constraint approximation's variable part at x(lam)
__global__ __launch_bounds__(RED_THREADS) void k_mma_eval(
    double lam, int64_t n, const double *__restrict__ low, const double *__restrict__ upp,
    const double *__restrict__ al, const double *__restrict__ be, const double *__restrict__ c,
    double *partial)
{
    double v[1] = {0.0};
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double xj = xlam(lam, c[4 * j], c[4 * j + 1], c[4 * j + 2], c[4 * j + 3], low[j],
                               upp[j], al[j], be[j]);
        v[0] += c[4 * j + 2] / (upp[j] - xj) + c[4 * j + 3] / (xj - low[j]);
    }
    mma_partials<1>(v, partial);
}

// history shift and the new iterate x(lam)
__global__ __launch_bounds__(256) void k_mma_final(double lam, int64_t n, double *__restrict__ x,
                                                   double *__restrict__ xold1,
                                                   double *__restrict__ xold2,
                                                   const double *__restrict__ low,
                                                   const double *__restrict__ upp,
                                                   const double *__restrict__ al,
                                                   const double *__restrict__ be,
                                                   const double *__restrict__ c)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double xj = x[j];
    xold2[j] = xold1[j];
    xold1[j] = xj;
    x[j] = xlam(lam, c[4 * j], c[4 * j + 1], c[4 * j + 2], c[4 * j + 3], low[j], upp[j], al[j],
                be[j]);
}

// ---- element-vector helpers of the optimisation loop ----------------------------

// out = design ? a : b
__global__ __launch_bounds__(256) void k_blend(int64_t n, const uint8_t *__restrict__ design,
                                               const double *__restrict__ a,
                                               const double *__restrict__ b, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = design[i] ? a[i] : b[i];
}

// out = design ? scale * a : 0   (a may be NULL: out = design ? scale : 0)
__global__ __launch_bounds__(256) void k_masked_scale(int64_t n, const uint8_t *__restrict__ design,
                                                      const double *__restrict__ a, double scale,
                                                      double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = design[i] ? scale * (a ? a[i] : 1.0) : 0.0;
}

__global__ __launch_bounds__(256) void k_gather(int64_t nd, const int64_t *__restrict__ idx,
                                                const double *__restrict__ full,
                                                double *__restrict__ compact)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nd) compact[i] = full[idx[i]];
}

__global__ __launch_bounds__(256) void k_scatter(int64_t nd, const int64_t *__restrict__ idx,
                                                 const double *__restrict__ compact,
                                                 double *__restrict__ full)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nd) full[idx[i]] = compact[i];
}

// partials of sum_design (1 - g)  and  of max |a - b| (second row)
__global__ __launch_bounds__(RED_THREADS) void k_vol_change(int64_t n, const uint8_t *__restrict__ design,
                                                            const double *__restrict__ g,
                                                            int64_t nd, const double *__restrict__ a,
                                                            const double *__restrict__ b,
                                                            double *partial)
{
    double v = 0.0, m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (design[i]) v += 1.0 - g[i];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nd;
         i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, fabs(a[i] - b[i]));
    __shared__ double red[2][RED_THREADS / 64];
    for (int o = 32; o > 0; o >>= 1) {
        v += __shfl_down(v, o, 64);
        m = fmax(m, __shfl_down(m, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = v;
        red[1][threadIdx.x >> 6] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0, mm = 0.0;
        for (int w = 0; w < RED_THREADS / 64; ++w) {
            s += red[0][w];
            mm = fmax(mm, red[1][w]);
        }
        partial[blockIdx.x] = s;
        partial[RED_BLOCKS + blockIdx.x] = mm;
    }
}

}  // namespace

inline unsigned nblk256(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_blend(int64_t n, const uint8_t *design, const double *a, const double *b,
                        double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_blend, dim3(nblk256(n)), dim3(256), 0, st, n, design, a, b, out);
    return hipGetLastError();
}

hipError_t launch_masked_scale(int64_t n, const uint8_t *design, const double *a, double scale,
                               double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_masked_scale, dim3(nblk256(n)), dim3(256), 0, st, n, design, a, scale, out);
    return hipGetLastError();
}

hipError_t launch_gather(int64_t nd, const int64_t *idx, const double *full, double *compact,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_gather, dim3(nblk256(nd)), dim3(256), 0, st, nd, idx, full, compact);
    return hipGetLastError();
}

hipError_t launch_scatter(int64_t nd, const int64_t *idx, const double *compact, double *full,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_scatter, dim3(nblk256(nd)), dim3(256), 0, st, nd, idx, compact, full);
    return hipGetLastError();
}

hipError_t launch_vol_change(int64_t n, const uint8_t *design, const double *g, int64_t nd,
                             const double *a, const double *b, double *partial, hipStream_t st)
{
    hipLaunchKernelGGL(k_vol_change, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, n, design, g, nd,
                       a, b, partial);
    return hipGetLastError();
}


hipError_t mma_alloc(MmaState *m)
{
    const size_t b = sizeof(double) * m->n;
    hipError_t e = hipMalloc(&m->xold1, b);
    if (e == hipSuccess) e = hipMalloc(&m->xold2, b);
    if (e == hipSuccess) e = hipMalloc(&m->low, b);
    if (e == hipSuccess) e = hipMalloc(&m->upp, b);
    if (e == hipSuccess) e = hipMalloc(&m->al, b);
    if (e == hipSuccess) e = hipMalloc(&m->be, b);
    if (e == hipSuccess) e = hipMalloc(&m->c, 4 * b);
    if (e == hipSuccess) e = hipMalloc(&m->partial, sizeof(double) * RED_BLOCKS);
    if (e == hipSuccess) e = hipMalloc(&m->sum, sizeof(double) * 2);
    if (e == hipSuccess) e = hipHostMalloc(&m->hsum, sizeof(double) * 2);
    if (e == hipSuccess) e = hipMemset(m->xold1, 0, b);  // never read before set; kept defined
    if (e == hipSuccess) e = hipMemset(m->xold2, 0, b);
    return e;
}

void mma_free(MmaState *m)
{
    for (double *q : {m->xold1, m->xold2, m->low, m->upp, m->al, m->be, m->c, m->partial, m->sum})
        if (q) (void)hipFree(q);
    if (m->hsum) (void)hipHostFree(m->hsum);
}

static int mma_sum(MmaState *m, hipStream_t st, double *out)
{
    FE_CHECK_HIP(launch_reduce(m->partial, 1, m->sum, nullptr, false, st));
    FE_CHECK_HIP(hipMemcpyAsync(m->hsum, m->sum, sizeof(double), hipMemcpyDeviceToHost, st));
    FE_CHECK_HIP(hipStreamSynchronize(st));
    *out = m->hsum[0];
    return FE_OK;
}

// One MMA iteration on x (device, in/out).  f1: constraint value at x; df0,
// df1: device gradients.  The objective value does not enter the update.
int mma_update(MmaState *m, double *x, const double *df0, double f1, const double *df1,
               double *lam_out, hipStream_t st)
{
    m->k += 1;
    MmaPar P{m->xmin, m->xmax, m->move, m->k <= 2 ? 1 : 0};
    const dim3 rb(RED_BLOCKS), rt(RED_THREADS);
    hipLaunchKernelGGL(k_mma_prep, rb, rt, 0, st, P, m->n, (const double *)x, df0, df1,
                       (const double *)m->xold1, (const double *)m->xold2, m->low, m->upp, m->al,
                       m->be, m->c, m->partial);
    FE_CHECK_HIP(hipGetLastError());
    double s0;
    int rc = mma_sum(m, st, &s0);
    if (rc) return rc;
    const double r1 = f1 - s0;
    auto g = [&](double lam, double *val) -> int {
        hipLaunchKernelGGL(k_mma_eval, rb, rt, 0, st, lam, m->n, (const double *)m->low,
                           (const double *)m->upp, (const double *)m->al, (const double *)m->be,
                           (const double *)m->c, m->partial);
        FE_CHECK_HIP(hipGetLastError());
        double s;
        int r = mma_sum(m, st, &s);
        *val = r1 + s;
        return r;
    };
    double g0, lam = 0.0;
    rc = g(0.0, &g0);
    if (rc) return rc;
    if (!std::isfinite(g0)) {
        set_error("mma: non-finite constraint approximation");
        return FE_ENAN;
    }
    if (g0 > 0.0) {
        double lo = 0.0, hi = 1.0, gv;
        while (true) {
            rc = g(hi, &gv);
            if (rc) return rc;
            if (!(gv > 0.0) || hi >= 1e30) break;
            lo = hi;
            hi *= 2.0;
        }
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            rc = g(mid, &gv);
            if (rc) return rc;
            if (gv > 0.0)
                lo = mid;
            else
                hi = mid;
        }
        lam = hi;
    }
    hipLaunchKernelGGL(k_mma_final, dim3((unsigned)((m->n + 255) / 256)), dim3(256), 0, st, lam,
                       m->n, x, m->xold1, m->xold2, (const double *)m->low, (const double *)m->upp,
                       (const double *)m->al, (const double *)m->be, (const double *)m->c);
    FE_CHECK_HIP(hipGetLastError());
    if (lam_out) *lam_out = lam;
    return FE_OK;
}

}  // namespace fe
