// Batched vector kernels and deterministic reductions of the lockstep Krylov
// engine: each launch covers the vectors of every problem in its table.
//
// A problem's reduction partials are laid out per column and chunk
// (partial[c nchunk + chunk]); the chunking depends only on the vector length,
// every chunk sums its entries in a fixed order (wave64 shuffles, then the four
// waves through LDS), and the partials of a column are added in a fixed tree
// order, so that a problem's dot products are bitwise the same whatever else
// is in the batch.
#include "fe_batch.h"

namespace fe {
namespace {

__device__ __forceinline__ double bwave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of one value per thread over the 256-thread workgroup (fixed order);
// the result is valid in thread 0.  red: 4 doubles of LDS per call site.
__device__ __forceinline__ double bblock_sum(double v, double *red)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v = bwave_sum(v);
    if (lane == 0) red[wv] = v;
    __syncthreads();
    const double s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(256) void kb_fill(const BFill *__restrict__ tab, const int *__restrict__ off,
                                               int n)
{
    const int e = batch_entry(off, n);
    const BFill &a = tab[e];
    const int64_t i = (int64_t)(blockIdx.x - (unsigned)off[e]) * 256 + threadIdx.x;
    if (i < a.n) a.p[i] = 0.0;
}

__global__ __launch_bounds__(256) void kb_cast(const BCast *__restrict__ tab, const int *__restrict__ off,
                                               int n)
{
    const int e = batch_entry(off, n);
    const BCast &a = tab[e];
    const int64_t i = (int64_t)(blockIdx.x - (unsigned)off[e]) * 256 + threadIdx.x;
    if (i < a.n) a.b[i] = (float)a.a[i];
}

__global__ __launch_bounds__(256) void kb_widen(const BWiden *__restrict__ tab,
                                                const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BWiden &a = tab[e];
    const int64_t i = (int64_t)(blockIdx.x - (unsigned)off[e]) * 256 + threadIdx.x;
    if (i < a.n) a.b[i] = (double)a.a[i];
}

__global__ __launch_bounds__(256) void kb_axpby(const BAxpby *__restrict__ tab,
                                                const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BAxpby &a = tab[e];
    const int64_t i = (int64_t)(blockIdx.x - (unsigned)off[e]) * 256 + threadIdx.x;
    if (i < a.n) a.y[i] = a.a * a.x[i] + a.b * a.y[i];
}

__global__ __launch_bounds__(256) void kb_scale(const BScale *__restrict__ tab,
                                                const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BScale &a = tab[e];
    const int64_t i = (int64_t)(blockIdx.x - (unsigned)off[e]) * 256 + threadIdx.x;
    if (i < a.n) a.y[i] = a.x[i] / a.s[0];
}

// x += sum_j y_j Z_j, the terms added in j order
template <typename Tz>
__global__ __launch_bounds__(256) void kb_comb(const BComb<Tz> *__restrict__ tab,
                                               const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BComb<Tz> &a = tab[e];
    const int64_t i = (int64_t)(blockIdx.x - (unsigned)off[e]) * 256 + threadIdx.x;
    if (i >= a.n) return;
    double acc = a.x[i];
    for (int j = 0; j < a.k; ++j) acc += a.y[j] * (double)a.Z[(int64_t)j * a.ld + i];
    a.x[i] = acc;
}

template <typename T>
__global__ __launch_bounds__(256) void kb_copy(const BCopy<T> *__restrict__ tab,
                                               const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BCopy<T> &a = tab[e];
    const int64_t i = (int64_t)(blockIdx.x - (unsigned)off[e]) * 256 + threadIdx.x;
    if (i < a.n) a.b[i] = a.a[i];
}

// Partials of <V_c, w> for the BDOT_GROUP columns c of group g (column k is
// <w, w> when norm), over chunk ch of the problem's vector.
__global__ __launch_bounds__(256) void kb_dots(const BDots *__restrict__ tab,
                                               const int *__restrict__ off, int n)
{
    __shared__ double red[BDOT_GROUP][4];
    const int e = batch_entry(off, n);
    const BDots &a = tab[e];
    const int lb = (int)blockIdx.x - off[e];
    const int ch = lb % a.nchunk, grp = lb / a.nchunk;
    const int c0 = grp * BDOT_GROUP;
    const int kc = a.k + (a.norm ? 1 : 0);
    double acc[BDOT_GROUP];
#pragma unroll
    for (int q = 0; q < BDOT_GROUP; ++q) acc[q] = 0.0;
    const int64_t base = (int64_t)ch * 256 * a.ept + threadIdx.x;
    for (int r = 0; r < a.ept; ++r) {
        const int64_t i = base + (int64_t)r * 256;
        if (i >= a.n) break;
        const double wi = a.w[i];
#pragma unroll
        for (int q = 0; q < BDOT_GROUP; ++q) {
            const int c = c0 + q;
            if (c < a.k)
                acc[q] += a.V[(int64_t)c * a.ld + i] * wi;
            else if (c < kc)
                acc[q] += wi * wi;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < BDOT_GROUP; ++q) {
        const double s = bwave_sum(acc[q]);
        if (lane == 0) red[q][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < BDOT_GROUP) {
        const int q = threadIdx.x, c = c0 + q;
        if (c < kc) a.partial[(int64_t)c * a.nchunk + ch] = (red[q][0] + red[q][1]) + (red[q][2] + red[q][3]);
    }
}

// One workgroup per column: the column's sum over its chunks (chunk order
// within each thread, then the fixed block order).
__global__ __launch_bounds__(256) void kb_reduce(const BReduce *__restrict__ tab,
                                                 const int *__restrict__ off, int n)
{
    __shared__ double red[4];
    const int e = batch_entry(off, n);
    const BReduce &a = tab[e];
    const int c = (int)blockIdx.x - off[e];
    double v = 0.0;
    for (int i = threadIdx.x; i < a.nchunk; i += 256) v += a.partial[(int64_t)c * a.nchunk + i];
    const double s = bblock_sum(v, red);
    if (threadIdx.x == 0) {
        a.out[c] = s;
        if (a.beta && c == a.ncol - 1) a.beta[0] = sqrt(s);
    }
}

// y = x / |x|: every workgroup adds the nchunk partials of |x|^2 in the same
// fixed order (so all see the same norm); workgroup 0 also stores |x|^2 and |x|.
__global__ __launch_bounds__(256) void kb_scale_norm(const BScaleNorm *__restrict__ tab,
                                                     const int *__restrict__ off, int n)
{
    __shared__ double red[4];
    const int e = batch_entry(off, n);
    const BScaleNorm &a = tab[e];
    const int lb = (int)blockIdx.x - off[e];
    double v = 0.0;
    for (int i = threadIdx.x; i < a.nchunk; i += 256) v += a.partial[i];
    const double s = bblock_sum(v, red);
    const double beta = sqrt(s);
    if (lb == 0 && threadIdx.x == 0) {
        a.nrm2[0] = s;
        a.beta[0] = beta;
    }
    const int64_t i = (int64_t)lb * 256 + threadIdx.x;
    if (i < a.n) a.y[i] = a.x[i] / beta;
}

// Reduction column of accumulator q of a group of nc basis columns from c0.
__device__ __forceinline__ int bdgs_out(int q, int nc, int w, int J, int c0)
{
    if (q < nc) return c0 + q;  // s
    q -= nc;
    if (w) {
        if (q < nc) return J + 1 + c0 + q;  // p
        q -= nc;
    }
    return q == 0 ? J : (q == 1 ? 2 * J + 1 : 2 * J + 2);  // a, t, e
}

// Partials of the delayed Gram-Schmidt dot products for the BDOT_GROUP basis
// columns of group g over chunk ch of the problem's vectors.
__global__ __launch_bounds__(256) void kb_dgs_dots(const BDgsDots *__restrict__ tab,
                                                   const int *__restrict__ off, int n)
{
    constexpr int G = BDOT_GROUP, NA = 2 * G + 3;
    __shared__ double red[NA][4];
    const int e = batch_entry(off, n);
    const BDgsDots &a = tab[e];
    const int lb = (int)blockIdx.x - off[e];
    const int ch = lb % a.nchunk, grp = lb / a.nchunk;
    const int c0 = grp * G;
    const int nc = min(G, a.J - c0);  // may be 0 (group 0 of J = 0)
    const double *__restrict__ c = a.V + (int64_t)a.J * a.ld;
    const double *__restrict__ w = a.V + (int64_t)(a.J + 1) * a.ld;
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    const int64_t base = (int64_t)ch * 256 * a.ept + threadIdx.x;
    for (int r = 0; r < a.ept; ++r) {
        const int64_t i = base + (int64_t)r * 256;
        if (i >= a.n) break;
        const double ci = c[i];
        const double wi = a.w ? w[i] : 0.0;
#pragma unroll
        for (int k = 0; k < G; ++k) {
            if (k < nc) {
                const double qk = a.V[(int64_t)(c0 + k) * a.ld + i];
                acc[k] += qk * ci;
                acc[G + k] += qk * wi;
            }
        }
        if (grp == 0) {
            acc[2 * G] += ci * ci;
            acc[2 * G + 1] += ci * wi;
            acc[2 * G + 2] += wi * wi;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const double s = bwave_sum(acc[q]);
        if (lane == 0) red[q][wv] = s;
    }
    __syncthreads();
    // the group's outputs in the order s (nc), p (nc, if w), then a, t, e (group 0)
    const int nout = nc * (a.w ? 2 : 1) + (grp == 0 ? (a.w ? 3 : 1) : 0);
    if ((int)threadIdx.x < nout) {
        const int q = threadIdx.x;
        int src;  // accumulator of output q
        if (q < nc)
            src = q;
        else if (a.w && q < 2 * nc)
            src = G + (q - nc);
        else
            src = 2 * G + (q - nc * (a.w ? 2 : 1));
        a.partial[(int64_t)bdgs_out(q, nc, a.w, a.J, c0) * a.nchunk + ch] =
            (red[src][0] + red[src][1]) + (red[src][2] + red[src][3]);
    }
}

// Update pass of delayed Gram-Schmidt over one chunk.  Every workgroup of a
// problem derives sigma = sqrt(a - |s|^2), h = (t - <s, p>) / sigma and
// omega = |w| from the reduced dot products in the same fixed order (wave 0,
// lane i holding s_i and p_i), so all use the same values; workgroup 0 stores
// them.
__global__ __launch_bounds__(256) void kb_dgs_update(const BDgsUpdate *__restrict__ tab,
                                                     const int *__restrict__ off, int n)
{
    __shared__ double cs[64], cp[64], coef[4];
    const int e = batch_entry(off, n);
    const BDgsUpdate &a = tab[e];
    const int ch = (int)blockIdx.x - off[e];
    const int J = a.J;
    if (threadIdx.x < 64) {
        const int l = threadIdx.x;
        const double sl = l < J ? a.res[l] : 0.0;
        const double pl = l < J ? a.res[J + 1 + l] : 0.0;
        cs[l] = sl;
        cp[l] = pl;
        const double ss = bwave_sum(sl * sl), sp = bwave_sum(sl * pl);
        const double s2 = a.res[J] - ss;
        const double sig = s2 > 0.0 ? sqrt(s2) : 0.0;
        const double h = sig > 0.0 ? (a.res[2 * J + 1] - sp) / sig : 0.0;
        const double om = sqrt(a.res[2 * J + 2]);
        if (l == 0) {
            coef[0] = sig > 0.0 ? 1.0 / sig : 0.0;
            coef[1] = h;
            coef[2] = om > 0.0 ? 1.0 / om : 0.0;
            if (ch == 0) {
                a.res[2 * J + 3] = sig;
                a.res[2 * J + 4] = h;
                a.res[2 * J + 5] = om;
            }
        }
    }
    __syncthreads();
    const double isg = coef[0], h = coef[1], iom = coef[2];
    double *__restrict__ c = a.V + (int64_t)J * a.ld;
    double *__restrict__ w = a.V + (int64_t)(J + 1) * a.ld;
    const double *__restrict__ Q = a.V;
    double acc = 0.0;
    const int64_t base = (int64_t)ch * 256 * a.ept + threadIdx.x;
    for (int r = 0; r < a.ept; ++r) {
        const int64_t i = base + (int64_t)r * 256;
        if (i >= a.n) break;
        double ci = c[i], wi = w[i];
        for (int k = 0; k < J; ++k) {
            const double qk = Q[(int64_t)k * a.ld + i];
            ci -= cs[k] * qk;
            wi -= cp[k] * qk;
        }
        const double qj = ci * isg;
        const double cn = (wi - h * qj) * iom;
        c[i] = qj;
        w[i] = cn;
        acc += cn * cn;
    }
    __shared__ double red[4];
    const double s = bblock_sum(acc, red);
    if (threadIdx.x == 0) a.partial[ch] = s;
}

}  // namespace

#define FE_BVLAUNCH(NAME, KERNEL, ARGS)                                                        \
    hipError_t NAME(const BLaunch &L, hipStream_t st)                                          \
    {                                                                                          \
        if (L.blocks <= 0) return hipSuccess;                                                  \
        hipLaunchKernelGGL(KERNEL, dim3((unsigned)L.blocks), dim3(256), 0, st,                 \
                           (const ARGS *)L.tab, L.off, L.n);                                    \
        return hipGetLastError();                                                              \
    }
FE_BVLAUNCH(blaunch_fill, kb_fill, BFill)
FE_BVLAUNCH(blaunch_cast, kb_cast, BCast)
FE_BVLAUNCH(blaunch_widen, kb_widen, BWiden)
FE_BVLAUNCH(blaunch_axpby, kb_axpby, BAxpby)
FE_BVLAUNCH(blaunch_scale, kb_scale, BScale)
FE_BVLAUNCH(blaunch_dots, kb_dots, BDots)
FE_BVLAUNCH(blaunch_reduce, kb_reduce, BReduce)
FE_BVLAUNCH(blaunch_dgs_dots, kb_dgs_dots, BDgsDots)
FE_BVLAUNCH(blaunch_dgs_update, kb_dgs_update, BDgsUpdate)
FE_BVLAUNCH(blaunch_scale_norm, kb_scale_norm, BScaleNorm)
#undef FE_BVLAUNCH

template <typename Tz>
hipError_t blaunch_comb(const BLaunch &L, hipStream_t st)
{
    if (L.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(kb_comb<Tz>, dim3((unsigned)L.blocks), dim3(256), 0, st,
                       (const BComb<Tz> *)L.tab, L.off, L.n);
    return hipGetLastError();
}
template hipError_t blaunch_comb<double>(const BLaunch &, hipStream_t);
template hipError_t blaunch_comb<float>(const BLaunch &, hipStream_t);

template <typename T>
hipError_t blaunch_copy(const BLaunch &L, hipStream_t st)
{
    if (L.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(kb_copy<T>, dim3((unsigned)L.blocks), dim3(256), 0, st,
                       (const BCopy<T> *)L.tab, L.off, L.n);
    return hipGetLastError();
}
template hipError_t blaunch_copy<double>(const BLaunch &, hipStream_t);
template hipError_t blaunch_copy<float>(const BLaunch &, hipStream_t);

}  // namespace fe
