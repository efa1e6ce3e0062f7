// Vector kernels of the Krylov / Newton loops on gfx950.
//
// Reductions are deterministic: a fixed grid of RED_BLOCKS workgroups each sums
// a fixed strided range (wave64 shuffles, then LDS across the four waves) into
// one partial per workgroup; a second kernel adds the partials in a fixed tree
// order.  Multi-dot products for classical Gram-Schmidt keep up to 64 running
// sums per thread in registers, so the basis vectors are streamed once per
// pass; the update w -= V h is fused with the next pass's dot products.
#include "fe_internal.h"

namespace fe {
namespace {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum KMAX per-thread accumulators over the workgroup; thread 0 writes them.
template <int KMAX>
__device__ __forceinline__ void block_sums(double (&acc)[KMAX], int k, double *partial)
{
    __shared__ double red[RED_THREADS / 64][KMAX];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        if (j < k) {
            double s = wave_sum(acc[j]);
            if (lane == 0) red[wv][j] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x < KMAX && (int)threadIdx.x < k) {
        const int j = threadIdx.x;
        double s = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
        partial[(int64_t)j * RED_BLOCKS + blockIdx.x] = s;
    }
}

template <int KMAX>
__global__ __launch_bounds__(RED_THREADS) void k_multidot(const double *__restrict__ V, int64_t ld,
                                                          int k, const double *__restrict__ w,
                                                          int64_t n, double *__restrict__ partial)
{
    double acc[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) acc[j] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double wi = w[i];
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < k) acc[j] += V[j * ld + i] * wi;
    }
    block_sums<KMAX>(acc, k, partial);
}

// w -= sum_{j<k} h[j] V_j; then partial <V_j, w> for j < k2, or <w, w> if k2 == -1.
template <int KMAX>
__global__ __launch_bounds__(RED_THREADS) void k_update_dot(const double *__restrict__ V, int64_t ld,
                                                            int k, const double *__restrict__ h,
                                                            double *__restrict__ w, int64_t n,
                                                            int k2, double *__restrict__ partial)
{
    __shared__ double hs[KMAX];
    if (threadIdx.x < KMAX && (int)threadIdx.x < k) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    double acc[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) acc[j] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double vj[KMAX];
        double wi = w[i];
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < k) {
                vj[j] = V[j * ld + i];
                wi -= hs[j] * vj[j];
            }
        w[i] = wi;
        if (k2 == -1) {
            acc[0] += wi * wi;
        } else {
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (j < k2) acc[j] += vj[j] * wi;
        }
    }
    if (partial) block_sums<KMAX>(acc, k2 == -1 ? 1 : k2, partial);
}

// Exact-count variants (K known at compile time, every load of an element
// issued together).  flag: optional device flag; the kernel does nothing
// when it is 0 (conditional second Gram-Schmidt pass).
template <int K, bool NORM>
__global__ __launch_bounds__(RED_THREADS) void k_mdot(const double *__restrict__ V, int64_t ld,
                                                      const double *__restrict__ w, int64_t n,
                                                      double *__restrict__ partial,
                                                      const double *__restrict__ flag)
{
    if (flag && flag[0] == 0.0) return;
    constexpr int KA = K + (NORM ? 1 : 0);
    double acc[KA];
#pragma unroll
    for (int j = 0; j < KA; ++j) acc[j] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double wi = w[i];
        double vj[K];
#pragma unroll
        for (int j = 0; j < K; ++j) vj[j] = V[j * ld + i];
#pragma unroll
        for (int j = 0; j < K; ++j) acc[j] += vj[j] * wi;
        if (NORM) acc[KA - 1] += wi * wi;
    }
    block_sums<KA>(acc, KA, partial);
}

template <int K>
__global__ __launch_bounds__(RED_THREADS) void k_upd(const double *__restrict__ V, int64_t ld,
                                                     const double *__restrict__ h,
                                                     double *__restrict__ w, int64_t n,
                                                     double *__restrict__ partial,
                                                     const double *__restrict__ flag)
{
    if (flag && flag[0] == 0.0) return;
    __shared__ double hs[K];
    if (threadIdx.x < K) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double vj[K];
#pragma unroll
        for (int j = 0; j < K; ++j) vj[j] = V[j * ld + i];
        double wi = w[i];
#pragma unroll
        for (int j = 0; j < K; ++j) wi -= hs[j] * vj[j];
        w[i] = wi;
        acc[0] += wi * wi;
    }
    block_sums<1>(acc, 1, partial);
}

// The first pass's update fused with the second pass's projection: w -= V h
// (h = V^T w from the first pass), then the partials of V^T w and |w|^2 of the
// updated w, in the same per-thread order as k_upd followed by k_mdot<K, true>,
// so V is read once for both.
template <int K>
__global__ __launch_bounds__(RED_THREADS) void k_upd_mdot(const double *__restrict__ V, int64_t ld,
                                                          const double *__restrict__ h,
                                                          double *__restrict__ w, int64_t n,
                                                          double *__restrict__ partial)
{
    __shared__ double hs[K];
    if (threadIdx.x < K) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    double acc[K + 1];
#pragma unroll
    for (int j = 0; j <= K; ++j) acc[j] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double vj[K];
#pragma unroll
        for (int j = 0; j < K; ++j) vj[j] = V[j * ld + i];
        double wi = w[i];
#pragma unroll
        for (int j = 0; j < K; ++j) wi -= hs[j] * vj[j];
        w[i] = wi;
#pragma unroll
        for (int j = 0; j < K; ++j) acc[j] += vj[j] * wi;
        acc[K] += wi * wi;
    }
    block_sums<K + 1>(acc, K + 1, partial);
}

// After the fused pass: flag = 1 when the projected norm beta1 fell below
// 1/sqrt(2) of the original norm (the second pass's update is needed), else 0,
// in which case the second-pass coefficients h2 are zeroed and beta = beta1.
// One wave (k <= 32): lane j zeroes h2[j], lane 0 writes the flag and beta.
__global__ void k_reorth_flag2(const double *__restrict__ w2_before, const double *__restrict__ beta1,
                               double *__restrict__ flag, double *__restrict__ h2, int k,
                               double *__restrict__ beta)
{
    const int t = threadIdx.x;
    const double nb = sqrt(w2_before[0]);
    const double b1 = beta1[0];
    const double again = (b1 < 0.70710678118654752 * nb) ? 1.0 : 0.0;
    if (t == 0) {
        flag[0] = again;
        if (again == 0.0) beta[0] = b1;
    }
    if (t < k && again == 0.0) h2[t] = 0.0;
}

__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ partial,
                                                double *__restrict__ out,
                                                const double *__restrict__ add, int k, int sqrt_last,
                                                const double *__restrict__ flag, int flag_mode,
                                                int nparts)
{
    // flag_mode 1: write zeros when *flag == 0; 2: leave out untouched when *flag == 0
    if (flag && flag[0] == 0.0) {
        if (flag_mode == 1 && threadIdx.x == 0) out[blockIdx.x] = 0.0;
        return;
    }
    // one workgroup per output; nparts (<= RED_BLOCKS) partials, summed in a
    // fixed tree: thread t adds partials t, t + 256, ... in order, then the waves
    __shared__ double red[4];
    const int j = blockIdx.x;
    const double *p = partial + (int64_t)j * RED_BLOCKS;
    double s = 0.0;
    for (int q = threadIdx.x; q < nparts; q += 256) s += p[q];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = (red[0] + red[1]) + (red[2] + red[3]);
        if (add) t += add[j];
        if (sqrt_last && j == k - 1) t = sqrt(t);
        out[j] = t;
    }
}

__global__ __launch_bounds__(RED_THREADS) void k_norm2_partial(const double *__restrict__ a,
                                                               int64_t n,
                                                               double *__restrict__ partial)
{
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        acc[0] += a[i] * a[i];
    block_sums<1>(acc, 1, partial);
}

__global__ void k_node_mask(const uint8_t *__restrict__ dm, uint8_t *__restrict__ nm, int64_t nn)
{
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    uint8_t m = 0;
    if (dm)
        for (int f = 0; f < NF; ++f)
            if (dm[NF * n + f]) m |= (uint8_t)(1u << f);
    nm[n] = m;
}

// In-place inverse of each 5x5 block by Gauss-Jordan with partial pivoting.
// The workgroup's 256 blocks pass through LDS both ways, so that global loads
// and stores are contiguous (a thread's block is 25 consecutive doubles; read
// and written directly, neighbouring lanes would touch addresses 200 B apart).
// Launched with 256 threads per workgroup.  T: the blocks' type and the
// arithmetic (D32, if given, receives an FP32 copy of FP64 inverses).
template <typename T>
__global__ __launch_bounds__(256) void k_invert_blocks(T *__restrict__ D, float *__restrict__ D32,
                                                       int64_t nn)
{
    __shared__ T sD[256 * 25];
    const int64_t n0 = (int64_t)blockIdx.x * 256;
    const T *Dn = stage_blocks256(D, n0, nn, sD);  // entries past nn: copies of the last
    T a[5][5], b[5][5];
#pragma unroll
    for (int r = 0; r < 5; ++r)
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            a[r][c] = Dn[r * 5 + c];
            b[r][c] = (r == c) ? T(1) : T(0);
        }
#pragma unroll
    for (int col = 0; col < 5; ++col) {
        int p = col;
        T best = fabs(a[col][col]);
#pragma unroll
        for (int r = col + 1; r < 5; ++r)
            if (fabs(a[r][col]) > best) {
                best = fabs(a[r][col]);
                p = r;
            }
#pragma unroll
        for (int r = col + 1; r < 5; ++r)
            if (r == p) {
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    T t = a[col][c]; a[col][c] = a[r][c]; a[r][c] = t;
                    t = b[col][c]; b[col][c] = b[r][c]; b[r][c] = t;
                }
            }
        const T inv = T(1) / a[col][col];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            a[col][c] *= inv;
            b[col][c] *= inv;
        }
#pragma unroll
        for (int r = 0; r < 5; ++r)
            if (r != col) {
                const T f = a[r][col];
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    a[r][c] -= f * a[col][c];
                    b[r][c] -= f * b[col][c];
                }
            }
    }
    // (every thread has read its own block above; it now overwrites only that)
    T *own = sD + threadIdx.x * 25;
#pragma unroll
    for (int r = 0; r < 5; ++r)
#pragma unroll
        for (int c = 0; c < 5; ++c) own[r * 5 + c] = b[r][c];
    __syncthreads();
    const int64_t left = nn - n0;
    const int cnt = (int)(left < 256 ? left : 256) * 25;
    T *dst = D + n0 * 25;
    float *dst32 = D32 ? D32 + n0 * 25 : nullptr;
#pragma unroll
    for (int k = 0; k < 25; ++k) {
        const int q = (int)threadIdx.x + 256 * k;
        if (q < cnt) {
            dst[q] = sD[q];
            if (dst32) dst32[q] = (float)sD[q];
        }
    }
}

// Launched with 256 threads per workgroup (the block staging assumes it).
template <typename Tm, typename Tin, typename Tout, bool TR>
__global__ __launch_bounds__(256) void k_block_apply(const Tm *__restrict__ D,
                                                     const Tin *__restrict__ v,
                                                     Tout *__restrict__ z, int64_t nn,
                                                     const double *__restrict__ scale)
{
    __shared__ Tm sD[256 * 25];
    const int64_t n0 = (int64_t)blockIdx.x * 256;
    const Tm *Dn = stage_blocks256(D, n0, nn, sD);
    const int64_t n = n0 + threadIdx.x;
    if (n >= nn) return;
    using Tc = Tm;
    Tc vv[5];
    const Tc sc = scale ? (Tc)(1.0 / scale[0]) : Tc(1);
#pragma unroll
    for (int f = 0; f < 5; ++f) vv[f] = (Tc)v[n * 5 + f] * sc;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        Tc acc = 0;
#pragma unroll
        for (int c = 0; c < 5; ++c) acc += (TR ? Dn[c * 5 + r] : Dn[r * 5 + c]) * vv[c];
        z[n * 5 + r] = (Tout)acc;
    }
}

__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b,
                        double *__restrict__ y)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // b == 0 overwrites y without reading it (y may hold anything, even NaN)
    y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}

__global__ void k_xpld(int64_t n, const double *__restrict__ x, double lam,
                       const double *__restrict__ d, double *__restrict__ y)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i] + lam * d[i];
}

__global__ void k_scale_div(int64_t n, const double *__restrict__ x, const double *__restrict__ s,
                            double *__restrict__ y)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double inv = 1.0 / s[0];
    if (i < n) y[i] = x[i] * inv;
}

template <typename Tz>
__global__ void k_combine_vec(const Tz *__restrict__ Z, int64_t ld, int k,
                              const double *__restrict__ c, double *__restrict__ y, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = y[i];
    for (int j = 0; j < k; ++j) acc += c[j] * (double)Z[j * ld + i];
    y[i] = acc;
}

template <typename Ta, typename Tb>
__global__ void k_cast(const Ta *__restrict__ a, Tb *__restrict__ b, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (Tb)a[i];
}

// Thermal compliance: c_n = sum over the node's source elements of s_e h^3/8;
// partial sums of T_n c_n; dfdx = c on unprescribed T entries.
__global__ __launch_bounds__(RED_THREADS) void k_compliance(Geo g, const double *__restrict__ x,
                                                            const double *__restrict__ s,
                                                            const uint8_t *__restrict__ nmask,
                                                            double *__restrict__ dfdx,
                                                            double *__restrict__ partial)
{
    const int64_t nn = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    const double w8 = 0.125 * g.h * g.h * g.h;
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += stride) {
        const int I = (int)(n % (g.nx + 1));
        const int64_t r = n / (g.nx + 1);
        const int J = (int)(r % (g.ny + 1));
        const int K = (int)(r / (g.ny + 1));
        double cn = 0.0;
        for (int dz = -1; dz <= 0; ++dz)
            for (int dy = -1; dy <= 0; ++dy)
                for (int dx = -1; dx <= 0; ++dx) {
                    int i = I + dx, j = J + dy, k = K + dz;
                    if (i < 0 || j < 0 || k < 0 || i >= g.nx || j >= g.ny || k >= g.nz) continue;
                    cn += s[i + (int64_t)g.nx * (j + (int64_t)g.ny * k)] * w8;
                }
        acc[0] += x[NF * n + 4] * cn;
        if (dfdx) {
            for (int f = 0; f < 4; ++f) dfdx[NF * n + f] = 0.0;
            dfdx[NF * n + 4] = ((nmask[n] >> 4) & 1) ? 0.0 : cn;
        }
    }
    block_sums<1>(acc, 1, partial);
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_node_mask(const uint8_t *dof_mask, uint8_t *nmask, int64_t nn, hipStream_t st)
{
    hipLaunchKernelGGL(k_node_mask, dim3(nblk(nn)), dim3(256), 0, st, dof_mask, nmask, nn);
    return hipGetLastError();
}

hipError_t launch_invert_blocks(double *D, float *D32, int64_t nn, hipStream_t st)
{
    hipLaunchKernelGGL(k_invert_blocks<double>, dim3(nblk(nn, 256)), dim3(256), 0, st, D, D32, nn);
    return hipGetLastError();
}

hipError_t launch_invert_blocks32(float *D32, int64_t nn, hipStream_t st)
{
    hipLaunchKernelGGL(k_invert_blocks<float>, dim3(nblk(nn, 256)), dim3(256), 0, st, D32,
                       (float *)nullptr, nn);
    return hipGetLastError();
}

template <typename Tm, typename Tin, typename Tout>
hipError_t launch_block_apply(const Tm *D, const Tin *v, Tout *z, int64_t nn, bool transpose,
                              const double *scale_dev, hipStream_t st)
{
    if (transpose)
        hipLaunchKernelGGL((k_block_apply<Tm, Tin, Tout, true>), dim3(nblk(nn)), dim3(256), 0, st,
                           D, v, z, nn, scale_dev);
    else
        hipLaunchKernelGGL((k_block_apply<Tm, Tin, Tout, false>), dim3(nblk(nn)), dim3(256), 0, st,
                           D, v, z, nn, scale_dev);
    return hipGetLastError();
}
template hipError_t launch_block_apply<double, double, double>(const double *, const double *,
                                                               double *, int64_t, bool,
                                                               const double *, hipStream_t);
template hipError_t launch_block_apply<float, double, float>(const float *, const double *, float *,
                                                             int64_t, bool, const double *,
                                                             hipStream_t);

hipError_t launch_multidot(const double *V, int64_t ld, int k, const double *w, int64_t n,
                           double *partial, hipStream_t st)
{
    if (k <= 8)
        hipLaunchKernelGGL(k_multidot<8>, dim3(red_blocks(n)), dim3(RED_THREADS), 0, st, V, ld, k, w, n, partial);
    else if (k <= 32)
        hipLaunchKernelGGL(k_multidot<32>, dim3(red_blocks(n)), dim3(RED_THREADS), 0, st, V, ld, k, w, n, partial);
    else
        hipLaunchKernelGGL(k_multidot<65>, dim3(red_blocks(n)), dim3(RED_THREADS), 0, st, V, ld, k, w, n, partial);
    return hipGetLastError();
}

hipError_t launch_update_dot(const double *V, int64_t ld, int k, const double *h, double *w,
                             int64_t n, int k2, double *partial, hipStream_t st)
{
    const int kk = k > k2 ? k : k2;
    if (kk <= 8)
        hipLaunchKernelGGL(k_update_dot<8>, dim3(red_blocks(n)), dim3(RED_THREADS), 0, st, V, ld, k, h, w, n, k2, partial);
    else if (kk <= 32)
        hipLaunchKernelGGL(k_update_dot<32>, dim3(red_blocks(n)), dim3(RED_THREADS), 0, st, V, ld, k, h, w, n, k2, partial);
    else
        hipLaunchKernelGGL(k_update_dot<65>, dim3(red_blocks(n)), dim3(RED_THREADS), 0, st, V, ld, k, h, w, n, k2, partial);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partial, int k, double *out, const double *add,
                         bool sqrt_last, hipStream_t st, int nparts)
{
    hipLaunchKernelGGL(k_reduce, dim3(k), dim3(256), 0, st, partial, out, add, k, sqrt_last ? 1 : 0,
                       (const double *)nullptr, 0, nparts);
    return hipGetLastError();
}

// Exact-count dispatch for 1 <= k <= 32.
#define FE_K_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) \
    X(14) X(15) X(16) X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) \
    X(29) X(30) X(31) X(32)

static hipError_t mdot_exact(int k, bool norm, const double *V, int64_t ld, const double *w,
                             int64_t n, double *partial, const double *flag, hipStream_t st)
{
    const dim3 g(red_blocks(n)), b(RED_THREADS);
    switch (k) {
#define FE_MD(K)                                                                               \
    case K:                                                                                    \
        if (norm)                                                                              \
            hipLaunchKernelGGL((k_mdot<K, true>), g, b, 0, st, V, ld, w, n, partial, flag);    \
        else                                                                                   \
            hipLaunchKernelGGL((k_mdot<K, false>), g, b, 0, st, V, ld, w, n, partial, flag);   \
        break;
        FE_K_CASES(FE_MD)
#undef FE_MD
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t upd_exact(int k, const double *V, int64_t ld, const double *h, double *w,
                            int64_t n, double *partial, const double *flag, hipStream_t st)
{
    const dim3 g(red_blocks(n)), b(RED_THREADS);
    switch (k) {
#define FE_UP(K)                                                                               \
    case K:                                                                                    \
        hipLaunchKernelGGL((k_upd<K>), g, b, 0, st, V, ld, h, w, n, partial, flag);            \
        break;
        FE_K_CASES(FE_UP)
#undef FE_UP
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t upd_mdot_exact(int k, const double *V, int64_t ld, const double *h, double *w,
                                 int64_t n, double *partial, hipStream_t st)
{
    const dim3 g(red_blocks(n)), b(RED_THREADS);
    switch (k) {
#define FE_UM(K)                                                                               \
    case K:                                                                                    \
        hipLaunchKernelGGL((k_upd_mdot<K>), g, b, 0, st, V, ld, h, w, n, partial);             \
        break;
        FE_K_CASES(FE_UM)
#undef FE_UM
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cgs(const double *V, int64_t ld, int k, double *w, int64_t n, double *hbuf,
                      double *partial, hipStream_t st)
{
    hipError_t e;
    const int np = red_blocks(n);
    if (k > 32) {  // long bases: unconditional two passes with the generic kernels
        if ((e = launch_multidot(V, ld, k, w, n, partial, st)) != hipSuccess) return e;
        if ((e = launch_reduce(partial, k, hbuf, nullptr, false, st, np)) != hipSuccess) return e;
        if ((e = launch_update_dot(V, ld, k, hbuf, w, n, k, partial, st)) != hipSuccess) return e;
        if ((e = launch_reduce(partial, k, hbuf + 65, nullptr, false, st, np)) != hipSuccess) return e;
        if ((e = launch_update_dot(V, ld, k, hbuf + 65, w, n, -1, partial, st)) != hipSuccess) return e;
        return launch_reduce(partial, 1, hbuf + 130, nullptr, true, st, np);
    }
    double *flag = hbuf + 131;
    // pass 1: h1 = V^T w and |w|^2 (stored at hbuf[k])
    if ((e = mdot_exact(k, true, V, ld, w, n, partial, nullptr, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce, dim3(k + 1), dim3(256), 0, st, partial, hbuf, (const double *)nullptr,
                       k + 1, 0, (const double *)nullptr, 0, np);
    // w -= V h1 and, in the same read of V, h2 = V^T w and beta1 = |w| (hbuf[65 + k])
    if ((e = upd_mdot_exact(k, V, ld, hbuf, w, n, partial, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce, dim3(k + 1), dim3(256), 0, st, partial, hbuf + 65,
                       (const double *)nullptr, k + 1, 1, (const double *)nullptr, 0, np);
    hipLaunchKernelGGL(k_reorth_flag2, dim3(1), dim3(64), 0, st, (const double *)(hbuf + k),
                       (const double *)(hbuf + 65 + k), flag, hbuf + 65, k, hbuf + 130);
    // the second pass's update only where the flag asks for it: w -= V h2, beta
    if ((e = upd_exact(k, V, ld, hbuf + 65, w, n, partial, flag, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, partial, hbuf + 130,
                       (const double *)nullptr, 1, 1, flag, 2, np);
    return hipGetLastError();
}

hipError_t launch_norm2_partial(const double *a, int64_t n, double *partial, hipStream_t st)
{
    hipLaunchKernelGGL(k_norm2_partial, dim3(red_blocks(n)), dim3(RED_THREADS), 0, st, a, n, partial);
    return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(256), 0, st, n, a, x, b, y);
    return hipGetLastError();
}

hipError_t launch_xpld(int64_t n, const double *x, double lam, const double *d, double *y,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_xpld, dim3(nblk(n)), dim3(256), 0, st, n, x, lam, d, y);
    return hipGetLastError();
}

hipError_t launch_scale_div(int64_t n, const double *x, const double *s, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_scale_div, dim3(nblk(n)), dim3(256), 0, st, n, x, s, y);
    return hipGetLastError();
}

template <typename Tz>
hipError_t launch_combine(const Tz *Z, int64_t ld, int k, const double *c, double *y, int64_t n,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_combine_vec<Tz>, dim3(nblk(n)), dim3(256), 0, st, Z, ld, k, c, y, n);
    return hipGetLastError();
}
template hipError_t launch_combine<double>(const double *, int64_t, int, const double *, double *,
                                           int64_t, hipStream_t);
template hipError_t launch_combine<float>(const float *, int64_t, int, const double *, double *,
                                          int64_t, hipStream_t);

template <typename Ta, typename Tb>
hipError_t launch_cast(const Ta *a, Tb *b, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL((k_cast<Ta, Tb>), dim3(nblk(n)), dim3(256), 0, st, a, b, n);
    return hipGetLastError();
}
template hipError_t launch_cast<double, float>(const double *, float *, int64_t, hipStream_t);
template hipError_t launch_cast<float, double>(const float *, double *, int64_t, hipStream_t);

hipError_t launch_compliance(const Geo &g, const double *x, const double *s, const uint8_t *nmask,
                             double *dfdx, double *partial, hipStream_t st)
{
    hipLaunchKernelGGL(k_compliance, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, g, x, s, nmask,
                       dfdx, partial);
    return hipGetLastError();
}

}  // namespace fe

namespace fe {
namespace {
// Walls (u, v, w, T on every boundary node) plus the pressure of node 0.
__global__ void k_wall_mask(int nx, int ny, int nz, uint8_t *__restrict__ nmask,
                            uint8_t *__restrict__ dof_mask)
{
    const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int I = (int)(n % (nx + 1));
    const int64_t r = n / (nx + 1);
    const int J = (int)(r % (ny + 1)), K = (int)(r / (ny + 1));
    const bool wall = I == 0 || J == 0 || K == 0 || I == nx || J == ny || K == nz;
    uint8_t m = wall ? (uint8_t)(1 | 2 | 4 | 16) : (uint8_t)0;
    if (n == 0) m |= 8;
    nmask[n] = m;
    for (int f = 0; f < NF; ++f) dof_mask[NF * n + f] = (m >> f) & 1;
}
}  // namespace

hipError_t launch_wall_mask(int nx, int ny, int nz, uint8_t *nmask, uint8_t *dof_mask, hipStream_t st)
{
    const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    hipLaunchKernelGGL(k_wall_mask, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, nx, ny, nz,
                       nmask, dof_mask);
    return hipGetLastError();
}
}  // namespace fe
