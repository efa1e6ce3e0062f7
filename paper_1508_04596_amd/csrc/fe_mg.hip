// Grid-transfer and smoothing kernels of the matrix-free geometric multigrid
// preconditioner (Sec. "Solving the linear systems": flexible GMRES with a
// geometric multigrid preconditioner; here the coarse operators are
// rediscretised on the coarse grid instead of formed by Galerkin projection,
// since no matrix is assembled).
//
// Coarse grids halve the element count in every direction; coarse node
// (I,J,K) coincides with fine node (2I,2J,2K).  Prolongation is trilinear
// interpolation, restriction its transpose (weights 1, 1/2, 1/4, 1/8).
#include "fe_internal.h"

namespace fe {
namespace {

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// coarse element = mean of its 8 children (design and source)
__global__ void k_coarsen_elem(int ncx, int ncy, int ncz, const double *__restrict__ f,
                               double *__restrict__ c)
{
    const int64_t nc = (int64_t)ncx * ncy * ncz;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nc) return;
    const int I = (int)(e % ncx);
    const int64_t r = e / ncx;
    const int J = (int)(r % ncy), K = (int)(r / ncy);
    const int nfx = 2 * ncx, nfy = 2 * ncy;
    double s = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                s += f[(2 * I + dx) + (int64_t)nfx * ((2 * J + dy) + (int64_t)nfy * (2 * K + dz))];
    c[e] = 0.125 * s;
}

// coarse node values taken from the coincident fine node (NV values per node)
template <typename Tf, typename Tc, int NV>
__global__ void k_inject(int ncx, int ncy, int ncz, const Tf *__restrict__ f, Tc *__restrict__ c)
{
    const int64_t nn = (int64_t)(ncx + 1) * (ncy + 1) * (ncz + 1);
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int I = (int)(n % (ncx + 1));
    const int64_t r = n / (ncx + 1);
    const int J = (int)(r % (ncy + 1)), K = (int)(r / (ncy + 1));
    const int nfx = 2 * ncx + 1, nfy = 2 * ncy + 1;
    const int64_t fn = (int64_t)(2 * I) + nfx * ((int64_t)(2 * J) + (int64_t)nfy * (2 * K));
#pragma unroll
    for (int q = 0; q < NV; ++q) c[NV * n + q] = (Tc)f[NV * fn + q];
}

// b_c = R (b - t) on unprescribed coarse DOFs, 0 on prescribed ones.
template <typename T>
__global__ void k_restrict(int ncx, int ncy, int ncz, const T *__restrict__ b,
                           const T *__restrict__ t, const uint8_t *__restrict__ cmask,
                           T *__restrict__ bc)
{
    const int64_t nn = (int64_t)(ncx + 1) * (ncy + 1) * (ncz + 1);
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int I = (int)(n % (ncx + 1));
    const int64_t r = n / (ncx + 1);
    const int J = (int)(r % (ncy + 1)), K = (int)(r / (ncy + 1));
    const int nfx = 2 * ncx, nfy = 2 * ncy, nfz = 2 * ncz;
    T acc[NF] = {T(0), T(0), T(0), T(0), T(0)};
    for (int dz = -1; dz <= 1; ++dz) {
        const int k = 2 * K + dz;
        if (k < 0 || k > nfz) continue;
        const T wz = dz == 0 ? T(1) : T(0.5);
        for (int dy = -1; dy <= 1; ++dy) {
            const int j = 2 * J + dy;
            if (j < 0 || j > nfy) continue;
            const T wy = dy == 0 ? T(1) : T(0.5);
            for (int dx = -1; dx <= 1; ++dx) {
                const int i = 2 * I + dx;
                if (i < 0 || i > nfx) continue;
                const T w = (dx == 0 ? T(1) : T(0.5)) * wy * wz;
                const int64_t fn = i + (int64_t)(nfx + 1) * (j + (int64_t)(nfy + 1) * k);
#pragma unroll
                for (int f = 0; f < NF; ++f) acc[f] += w * (b[NF * fn + f] - (t ? t[NF * fn + f] : T(0)));
            }
        }
    }
    const uint8_t m = cmask[n];
#pragma unroll
    for (int f = 0; f < NF; ++f) bc[NF * n + f] = ((m >> f) & 1) ? T(0) : acc[f];
}

// x += P xc on unprescribed fine DOFs (trilinear interpolation).
template <typename T>
__global__ void k_prolong_add(int nfx, int nfy, int nfz, const T *__restrict__ xc,
                              const uint8_t *__restrict__ fmask, T *__restrict__ x)
{
    const int64_t nn = (int64_t)(nfx + 1) * (nfy + 1) * (nfz + 1);
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int i = (int)(n % (nfx + 1));
    const int64_t r = n / (nfx + 1);
    const int j = (int)(r % (nfy + 1)), k = (int)(r / (nfy + 1));
    const int ncx = nfx / 2, ncy = nfy / 2;
    int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
    const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (k & 1) ? 2 : 1;
    const T wi = ni == 2 ? T(0.5) : T(1), wj = nj == 2 ? T(0.5) : T(1), wk = nk == 2 ? T(0.5) : T(1);
    T acc[NF] = {T(0), T(0), T(0), T(0), T(0)};
    for (int c = 0; c < nk; ++c)
        for (int bq = 0; bq < nj; ++bq)
            for (int a = 0; a < ni; ++a) {
                const int64_t cn = (I0 + a) + (int64_t)(ncx + 1) * ((J0 + bq) + (int64_t)(ncy + 1) * (K0 + c));
#pragma unroll
                for (int f = 0; f < NF; ++f) acc[f] += xc[NF * cn + f];
            }
    const T w = wi * wj * wk;
    const uint8_t m = fmask[n];
#pragma unroll
    for (int f = 0; f < NF; ++f)
        if (!((m >> f) & 1)) x[NF * n + f] += w * acc[f];
}

// x (+)= omega * D^{-1} (b - t) per node (D^{-T} when TR); t may be NULL (= 0);
// ACC = false overwrites x.
template <typename T, bool TR, bool ACC>
__global__ void k_smooth(const T *__restrict__ D, const T *__restrict__ b, const T *__restrict__ t,
                         T *__restrict__ x, int64_t nn, T omega)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    T r[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) r[f] = b[NF * n + f] - (t ? t[NF * n + f] : T(0));
#pragma unroll
    for (int a = 0; a < NF; ++a) {
        T acc = T(0);
#pragma unroll
        for (int c = 0; c < NF; ++c) acc += (TR ? D[n * 25 + c * NF + a] : D[n * 25 + a * NF + c]) * r[c];
        if (ACC)
            x[NF * n + a] += omega * acc;
        else
            x[NF * n + a] = omega * acc;
    }
}

}  // namespace

hipError_t mg_coarsen_elem(int ncx, int ncy, int ncz, const double *f, double *c, hipStream_t st)
{
    const int64_t n = (int64_t)ncx * ncy * ncz;
    hipLaunchKernelGGL(k_coarsen_elem, dim3(nblk(n)), dim3(256), 0, st, ncx, ncy, ncz, f, c);
    return hipGetLastError();
}

hipError_t mg_inject_state(int ncx, int ncy, int ncz, const double *f, double *c, hipStream_t st)
{
    const int64_t n = (int64_t)(ncx + 1) * (ncy + 1) * (ncz + 1);
    hipLaunchKernelGGL((k_inject<double, double, NF>), dim3(nblk(n)), dim3(256), 0, st, ncx, ncy,
                       ncz, f, c);
    return hipGetLastError();
}

hipError_t mg_inject_mask(int ncx, int ncy, int ncz, const uint8_t *f, uint8_t *c, hipStream_t st)
{
    const int64_t n = (int64_t)(ncx + 1) * (ncy + 1) * (ncz + 1);
    hipLaunchKernelGGL((k_inject<uint8_t, uint8_t, 1>), dim3(nblk(n)), dim3(256), 0, st, ncx, ncy,
                       ncz, f, c);
    return hipGetLastError();
}

template <typename T>
hipError_t mg_restrict(int ncx, int ncy, int ncz, const T *b, const T *t, const uint8_t *cmask,
                       T *bc, hipStream_t st)
{
    const int64_t n = (int64_t)(ncx + 1) * (ncy + 1) * (ncz + 1);
    hipLaunchKernelGGL(k_restrict<T>, dim3(nblk(n)), dim3(256), 0, st, ncx, ncy, ncz, b, t, cmask, bc);
    return hipGetLastError();
}

template <typename T>
hipError_t mg_prolong_add(int nfx, int nfy, int nfz, const T *xc, const uint8_t *fmask, T *x,
                          hipStream_t st)
{
    const int64_t n = (int64_t)(nfx + 1) * (nfy + 1) * (nfz + 1);
    hipLaunchKernelGGL(k_prolong_add<T>, dim3(nblk(n)), dim3(256), 0, st, nfx, nfy, nfz, xc, fmask, x);
    return hipGetLastError();
}

template <typename T>
hipError_t mg_smooth(const T *D, const T *b, const T *t, T *x, int64_t nn, T omega, bool transpose,
                     bool accumulate, hipStream_t st)
{
    const dim3 g(nblk(nn)), bl(256);
    if (transpose) {
        if (accumulate)
            hipLaunchKernelGGL((k_smooth<T, true, true>), g, bl, 0, st, D, b, t, x, nn, omega);
        else
            hipLaunchKernelGGL((k_smooth<T, true, false>), g, bl, 0, st, D, b, t, x, nn, omega);
    } else {
        if (accumulate)
            hipLaunchKernelGGL((k_smooth<T, false, true>), g, bl, 0, st, D, b, t, x, nn, omega);
        else
            hipLaunchKernelGGL((k_smooth<T, false, false>), g, bl, 0, st, D, b, t, x, nn, omega);
    }
    return hipGetLastError();
}

#define FE_MG_INST(T)                                                                          \
    template hipError_t mg_restrict<T>(int, int, int, const T *, const T *, const uint8_t *, T *,  \
                                       hipStream_t);                                           \
    template hipError_t mg_prolong_add<T>(int, int, int, const T *, const uint8_t *, T *,        \
                                          hipStream_t);                                        \
    template hipError_t mg_smooth<T>(const T *, const T *, const T *, T *, int64_t, T, bool, bool, \
                                     hipStream_t);
FE_MG_INST(double)
FE_MG_INST(float)
#undef FE_MG_INST

}  // namespace fe
