// PDE (Helmholtz) density filter on the element grid (Sec. "Optimisation
// problem": the design field is regularised by a PDE-based density filter).
//
//   -r^2 lap(psi) + psi = gamma,  zero normal derivative on the box boundary,
//
// psi trilinear on the nodes, gamma constant per element, r = R / (2 sqrt 3).
// Filtered element value = mean of psi over the element's nodes:
//   F gamma = A K^-1 T gamma,  F^T g = T^T K^-1 A^T g,  K = r^2 K_lap + M.
// K is applied matrix-free node by node (each node sums the element matrix rows
// of its up to 8 elements; the element matrix depends only on the Hamming
// distance between the two corners), and K psi = b is solved by Jacobi-
// preconditioned conjugate gradients with every scalar kept on the device.
#include <cstring>

#include "fe_topopt.h"

namespace fe {
namespace {

__device__ __forceinline__ int64_t fnode(const FGeo &g, int I, int J, int K)
{
    return (int64_t)I + (int64_t)(g.nx + 1) * ((int64_t)J + (int64_t)(g.ny + 1) * K);
}

// y = K x at node n; also the node's number of elements (for the diagonal)
__device__ __forceinline__ double kapply(const FGeo &g, const double *__restrict__ x, int I, int J,
                                         int K, int *nel)
{
    double acc = 0.0;
    int cnt = 0;
    for (int ez = K - 1; ez <= K; ++ez) {
        if (ez < 0 || ez >= g.nz) continue;
        for (int ey = J - 1; ey <= J; ++ey) {
            if (ey < 0 || ey >= g.ny) continue;
            for (int ex = I - 1; ex <= I; ++ex) {
                if (ex < 0 || ex >= g.nx) continue;
                ++cnt;
                const int ca = (I - ex) | ((J - ey) << 1) | ((K - ez) << 2);
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int d = __popc(ca ^ b);
                    acc += g.E[d] * x[fnode(g, ex + (b & 1), ey + ((b >> 1) & 1), ez + (b >> 2))];
                }
            }
        }
    }
    *nel = cnt;
    return acc;
}

__device__ __forceinline__ void node_ijk(const FGeo &g, int64_t n, int &I, int &J, int &K)
{
    I = (int)(n % (g.nx + 1));
    const int64_t r = n / (g.nx + 1);
    J = (int)(r % (g.ny + 1));
    K = (int)(r / (g.ny + 1));
}

__device__ __forceinline__ int node_nel(const FGeo &g, int I, int J, int K)
{
    const int cx = (I > 0) + (I < g.nx), cy = (J > 0) + (J < g.ny), cz = (K > 0) + (K < g.nz);
    return cx * cy * cz;
}

// block partial sums over a grid-stride loop: partial[j * RED_BLOCKS + blockIdx.x]
template <int NV>
__device__ __forceinline__ void block_partials(double v[NV], double *partial)
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

// node value = scale * sum of the element values around the node (T: h^3/8; A^T: 1/8)
__global__ __launch_bounds__(256) void k_elem_to_node(FGeo g, const double *__restrict__ e,
                                                      double scale, double *__restrict__ out)
{
    const int64_t nn = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    int I, J, K;
    node_ijk(g, n, I, J, K);
    double acc = 0.0;
    for (int ez = K - 1; ez <= K; ++ez) {
        if (ez < 0 || ez >= g.nz) continue;
        for (int ey = J - 1; ey <= J; ++ey) {
            if (ey < 0 || ey >= g.ny) continue;
            for (int ex = I - 1; ex <= I; ++ex) {
                if (ex < 0 || ex >= g.nx) continue;
                acc += e[ex + (int64_t)g.nx * (ey + (int64_t)g.ny * ez)];
            }
        }
    }
    out[n] = scale * acc;
}

// element value = scale * sum of its 8 node values (A: 1/8; T^T: h^3/8)
__global__ __launch_bounds__(256) void k_node_to_elem(FGeo g, const double *__restrict__ nv,
                                                      double scale, double *__restrict__ out)
{
    const int64_t ne = (int64_t)g.nx * g.ny * g.nz;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((int64_t)g.nx * g.ny));
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < 8; ++b) acc += nv[fnode(g, i + (b & 1), j + ((b >> 1) & 1), k + (b >> 2))];
    out[e] = scale * acc;
}

// CG start from x = 0: r = b, z = D^-1 b, p = z; partials of <r, z> and <r, r>
__global__ __launch_bounds__(RED_THREADS) void k_cg_init(FGeo g, const double *__restrict__ b,
                                                         double *__restrict__ x, double *__restrict__ r,
                                                         double *__restrict__ p, double *partial)
{
    const int64_t nn = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    double v[2] = {0.0, 0.0};
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn;
         n += (int64_t)gridDim.x * blockDim.x) {
        int I, J, K;
        node_ijk(g, n, I, J, K);
        const double rn = b[n], zn = rn / (node_nel(g, I, J, K) * g.E[0]);
        x[n] = 0.0;
        r[n] = rn;
        p[n] = zn;
        v[0] += rn * zn;
        v[1] += rn * rn;
    }
    block_partials<2>(v, partial);
}

// y = K p, partials of <p, y>
__global__ __launch_bounds__(RED_THREADS) void k_cg_apply(FGeo g, const double *__restrict__ p,
                                                          double *__restrict__ y, double *partial)
{
    const int64_t nn = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    double v[1] = {0.0};
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn;
         n += (int64_t)gridDim.x * blockDim.x) {
        int I, J, K, nel;
        node_ijk(g, n, I, J, K);
        const double yn = kapply(g, p, I, J, K, &nel);
        y[n] = yn;
        v[0] += p[n] * yn;
    }
    block_partials<1>(v, partial);
}

// alpha = rz / pAp; x += alpha p; r -= alpha y; partials of <r, D^-1 r> and <r, r>
__global__ __launch_bounds__(RED_THREADS) void k_cg_step(FGeo g, const double *__restrict__ sc,
                                                         int cur, const double *__restrict__ p,
                                                         const double *__restrict__ y,
                                                         double *__restrict__ x,
                                                         double *__restrict__ r, double *partial)
{
    const int64_t nn = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    const double alpha = sc[cur] / sc[2];  // rz / pAp
    double v[2] = {0.0, 0.0};
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn;
         n += (int64_t)gridDim.x * blockDim.x) {
        int I, J, K;
        node_ijk(g, n, I, J, K);
        x[n] += alpha * p[n];
        const double rn = r[n] - alpha * y[n];
        r[n] = rn;
        v[0] += rn * rn / (node_nel(g, I, J, K) * g.E[0]);
        v[1] += rn * rn;
    }
    block_partials<2>(v, partial);
}

// beta = rz_new / rz_old; p = D^-1 r + beta p
__global__ __launch_bounds__(256) void k_cg_dir(FGeo g, const double *__restrict__ sc, int cur,
                                                const double *__restrict__ r, double *__restrict__ p)
{
    const int64_t nn = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const double beta = sc[1 - cur] / sc[cur];  // new / old
    int I, J, K;
    node_ijk(g, n, I, J, K);
    p[n] = r[n] / (node_nel(g, I, J, K) * g.E[0]) + beta * p[n];
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// ---- host side --------------------------------------------------------------------


hipError_t filter_alloc(Filter *f, const fe_grid &grid, double radius)
{
    const double h = grid.h, r = radius / (2.0 * 1.7320508075688772935);
    const double kap[4] = {1.0 / 3.0, 0.0, -1.0 / 12.0, -1.0 / 12.0};
    const double mu[4] = {8.0, 4.0, 2.0, 1.0};
    f->g.nx = grid.nx;
    f->g.ny = grid.ny;
    f->g.nz = grid.nz;
    for (int d = 0; d < 4; ++d) f->g.E[d] = r * r * h * kap[d] + h * h * h / 216.0 * mu[d];
    f->nn = (int64_t)(grid.nx + 1) * (grid.ny + 1) * (grid.nz + 1);
    f->ne = (int64_t)grid.nx * grid.ny * grid.nz;
    f->load = h * h * h / 8.0;
    const size_t nb = sizeof(double) * f->nn;
    hipError_t e = hipMalloc(&f->b, nb);
    if (e == hipSuccess) e = hipMalloc(&f->x, nb);
    if (e == hipSuccess) e = hipMalloc(&f->r, nb);
    if (e == hipSuccess) e = hipMalloc(&f->p, nb);
    if (e == hipSuccess) e = hipMalloc(&f->y, nb);
    if (e == hipSuccess) e = hipMalloc(&f->partial, sizeof(double) * 2 * RED_BLOCKS);
    if (e == hipSuccess) e = hipMalloc(&f->sc, sizeof(double) * 8);
    if (e == hipSuccess) e = hipHostMalloc(&f->hsc, sizeof(double) * 8);
    return e;
}

void filter_free(Filter *f)
{
    for (double *q : {f->b, f->x, f->r, f->p, f->y, f->partial, f->sc})
        if (q) (void)hipFree(q);
    if (f->hsc) (void)hipHostFree(f->hsc);
}

// psi = K^-1 b (b, psi: the filter's own node buffers b and x); returns FE_OK,
// FE_NOT_CONVERGED or an error
int filter_solve(Filter *f, hipStream_t st, double rtol, int max_its)
{
    const FGeo &g = f->g;
    const dim3 rb(RED_BLOCKS), rt(RED_THREADS);
    hipLaunchKernelGGL(k_cg_init, rb, rt, 0, st, g, (const double *)f->b, f->x, f->r, f->p,
                       f->partial);
    // sc[0] = rz, sc[3] = rr; rr0 kept in sc[4]
    FE_CHECK_HIP(launch_reduce(f->partial, 1, f->sc + 0, nullptr, false, st));
    FE_CHECK_HIP(launch_reduce(f->partial + RED_BLOCKS, 1, f->sc + 4, nullptr, false, st));
    FE_CHECK_HIP(hipMemcpyAsync(f->hsc + 4, f->sc + 4, sizeof(double), hipMemcpyDeviceToHost, st));
    FE_CHECK_HIP(hipStreamSynchronize(st));
    const double rr0 = f->hsc[4];
    f->last_its = 0;
    if (!(rr0 > 0.0)) return rr0 == 0.0 ? FE_OK : FE_ENAN;
    int cur = 0;
    for (int it = 1; it <= max_its; ++it) {
        hipLaunchKernelGGL(k_cg_apply, rb, rt, 0, st, g, (const double *)f->p, f->y, f->partial);
        FE_CHECK_HIP(launch_reduce(f->partial, 1, f->sc + 2, nullptr, false, st));
        hipLaunchKernelGGL(k_cg_step, rb, rt, 0, st, g, (const double *)f->sc, cur,
                           (const double *)f->p, (const double *)f->y, f->x, f->r, f->partial);
        FE_CHECK_HIP(launch_reduce(f->partial, 1, f->sc + (1 - cur), nullptr, false, st));
        FE_CHECK_HIP(launch_reduce(f->partial + RED_BLOCKS, 1, f->sc + 3, nullptr, false, st));
        hipLaunchKernelGGL(k_cg_dir, dim3(nblk(f->nn)), dim3(256), 0, st, g, (const double *)f->sc,
                           cur, (const double *)f->r, f->p);
        FE_CHECK_HIP(hipGetLastError());
        cur = 1 - cur;
        f->last_its = it;
        if (it % 8 == 0 || it == max_its) {
            FE_CHECK_HIP(hipMemcpyAsync(f->hsc + 3, f->sc + 3, sizeof(double),
                                        hipMemcpyDeviceToHost, st));
            FE_CHECK_HIP(hipStreamSynchronize(st));
            const double rr = f->hsc[3];
            if (!std::isfinite(rr)) return FE_ENAN;
            if (rr <= rtol * rtol * rr0) return FE_OK;
        }
    }
    return FE_NOT_CONVERGED;
}

hipError_t filter_load(Filter *f, const double *gamma, double scale, hipStream_t st)
{
    hipLaunchKernelGGL(k_elem_to_node, dim3(nblk(f->nn)), dim3(256), 0, st, f->g, gamma, scale, f->b);
    return hipGetLastError();
}

hipError_t filter_unload(Filter *f, double scale, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_node_to_elem, dim3(nblk(f->ne)), dim3(256), 0, st, f->g,
                       (const double *)f->x, scale, out);
    return hipGetLastError();
}

}  // namespace fe
