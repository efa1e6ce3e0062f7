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

// w -= sum_{c<k} h_c V_c over one chunk, then (optionally) the chunk's <w, w>.
__global__ __launch_bounds__(256) void kb_update(const BUpdate *__restrict__ tab,
                                                 const int *__restrict__ off, int n)
{
    __shared__ double hs[BCOMB_MAX + 1];
    __shared__ double red[4];
    const int e = batch_entry(off, n);
    const BUpdate &a = tab[e];
    const int ch = (int)blockIdx.x - off[e];
    if ((int)threadIdx.x < a.k) hs[threadIdx.x] = a.h[threadIdx.x];
    __syncthreads();
    double acc = 0.0;
    const int64_t base = (int64_t)ch * 256 * a.ept + threadIdx.x;
    for (int r = 0; r < a.ept; ++r) {
        const int64_t i = base + (int64_t)r * 256;
        if (i >= a.n) break;
        double wi = a.w[i];
        for (int c = 0; c < a.k; ++c) wi -= hs[c] * a.V[(int64_t)c * a.ld + i];
        a.w[i] = wi;
        acc += wi * wi;
    }
    if (a.partial) {
        const double s = bblock_sum(acc, red);
        if (threadIdx.x == 0) a.partial[ch] = s;
    }
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
FE_BVLAUNCH(blaunch_axpby, kb_axpby, BAxpby)
FE_BVLAUNCH(blaunch_scale, kb_scale, BScale)
FE_BVLAUNCH(blaunch_dots, kb_dots, BDots)
FE_BVLAUNCH(blaunch_reduce, kb_reduce, BReduce)
FE_BVLAUNCH(blaunch_update, kb_update, BUpdate)
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
