// Vector kernels of the Krylov / Newton loops on gfx950.
//
// Reductions are deterministic: a fixed grid of RED_BLOCKS workgroups each sums
// a fixed strided range (wave64 shuffles, then LDS across the four waves) into
// one partial per workgroup; a second kernel adds the partials in a fixed tree
// order.  Gram-Schmidt is classical with the second projection of each basis
// vector delayed into the next step, so that a step streams the basis twice:
// one pass for all its dot products, one for the updates.
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

// ---- delayed classical Gram-Schmidt ---------------------------------------
// A step with J final basis vectors q_0 .. q_{J-1} (columns 0 .. J-1 of V),
// the candidate c (column J: the previous Krylov vector after one projection,
// scaled) and the new Krylov vector w (column J + 1) streams V twice.  The dot
// pass forms, as reduction columns of `partial`,
//   s_i = <q_i, c> at i (i < J), a = <c, c> at J, p_i = <q_i, w> at J + 1 + i,
//   t = <c, w> at 2J + 1, e = <w, w> at 2J + 2,
// so the candidate's second projection and w's first one share one read of
// the basis; the update pass then writes q_J = (c - sum s_i q_i) / sigma and
// the next candidate (w - sum p_i q_i - h q_J) / omega, with sigma, h and omega
// derived from the dot products.  A launch covers at most DGS_GROUP basis
// columns; the group that
// starts at column 0 also accumulates a, t and e.
//
// Both passes run RED_BLOCKS workgroups of 4 waves, at most 4 waves per SIMD,
// so their register budget is 128 VGPRs (DGS_WAVES).  Left to aim at 8 waves
// (64 VGPRs), the compiler fits the per-thread accumulators by reusing one
// load register and waits for each basis column's load before issuing the
// next: the dot pass then ran at 3.2-3.9 TB/s from 8 columns on.  With the
// budget stated, a group of up to 18 columns issues all its loads before the
// first wait, and no instantiation spills.
constexpr int DGS_GROUP = 32;
#define DGS_WAVES __attribute__((amdgpu_waves_per_eu(1, 4)))

// Reduction column of accumulator q of a group of nc columns from c0.
__device__ __forceinline__ int dgs_out(int q, int nc, bool w, int J, int c0)
{
    if (q < nc) return c0 + q;  // s
    q -= nc;
    if (w) {
        if (q < nc) return J + 1 + c0 + q;  // p
        q -= nc;
    }
    return q == 0 ? J : (q == 1 ? 2 * J + 1 : 2 * J + 2);  // a, t, e
}

template <int NC, bool W, bool FIRST>
__global__ __launch_bounds__(RED_THREADS) DGS_WAVES void k_dgs_dots(const double *__restrict__ V, int64_t ld,
                                                          int J, int c0, int64_t n,
                                                          double *__restrict__ partial)
{
    constexpr int NS = NC * (W ? 2 : 1);
    constexpr int NA = NS + (FIRST ? (W ? 3 : 1) : 0);
    const double *__restrict__ c = V + (int64_t)J * ld;
    const double *__restrict__ w = V + (int64_t)(J + 1) * ld;
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double ci = c[i];
        const double wi = W ? w[i] : 0.0;
        double qv[NC > 0 ? NC : 1];
#pragma unroll
        for (int k = 0; k < NC; ++k) qv[k] = V[(int64_t)(c0 + k) * ld + i];
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] += qv[k] * ci;
        if (W) {
#pragma unroll
            for (int k = 0; k < NC; ++k) acc[NC + k] += qv[k] * wi;
        }
        if (FIRST) {
            acc[NS] += ci * ci;
            if (W) {
                acc[NS + 1] += ci * wi;
                acc[NS + 2] += wi * wi;
            }
        }
    }
    __shared__ double red[RED_THREADS / 64][NA];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < NA) {
        const int q = threadIdx.x;
        partial[(int64_t)dgs_out(q, NC, W, J, c0) * RED_BLOCKS + blockIdx.x] =
            (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    }
}

// Update pass over the basis columns c0 .. c0 + NC - 1: c -= sum s_i q_i and
// w -= sum p_i q_i.  FINAL (the last group): then q_J = c / sigma into column
// J, the next candidate (w - h q_J) / omega into column J + 1, and the
// partials of its squared norm, where sigma = sqrt(a - |s|^2) (the candidate's
// norm after its second projection; 0 when nothing is left of it), h =
// (t - <s, p>) / sigma (the coefficient of w on q_J) and omega = |w| come from
// the reduced dot products in hb: every workgroup derives them in the same
// fixed order (wave 0, lane i holding s_i and p_i), and workgroup 0 stores
// them at hb[2J + 3 .. 2J + 5].  Columns below J are only read, so the three
// pointers never address the same entries; J <= 63.
template <int NC, bool FINAL>
__global__ __launch_bounds__(RED_THREADS) DGS_WAVES void k_dgs_update(const double *__restrict__ Q, double *__restrict__ c,
                                                            double *__restrict__ w, int64_t ld, int J,
                                                            int c0, int64_t n,
                                                            double *__restrict__ hb,
                                                            double *__restrict__ partial)
{
    __shared__ double cs[NC > 0 ? NC : 1], cp[NC > 0 ? NC : 1], coef[3];
    if ((int)threadIdx.x < NC) {
        cs[threadIdx.x] = hb[c0 + threadIdx.x];
        cp[threadIdx.x] = hb[J + 1 + c0 + threadIdx.x];
    }
    if (FINAL && threadIdx.x < 64) {
        const int l = threadIdx.x;
        const double sl = l < J ? hb[l] : 0.0;
        const double pl = l < J ? hb[J + 1 + l] : 0.0;
        const double ss = wave_sum(sl * sl), sp = wave_sum(sl * pl);
        const double s2 = hb[J] - ss;
        const double sig = s2 > 0.0 ? sqrt(s2) : 0.0;
        const double h = sig > 0.0 ? (hb[2 * J + 1] - sp) / sig : 0.0;
        const double om = sqrt(hb[2 * J + 2]);
        if (l == 0) {
            coef[0] = sig > 0.0 ? 1.0 / sig : 0.0;
            coef[1] = h;
            coef[2] = om > 0.0 ? 1.0 / om : 0.0;
            if (blockIdx.x == 0) {
                hb[2 * J + 3] = sig;
                hb[2 * J + 4] = h;
                hb[2 * J + 5] = om;
            }
        }
    }
    __syncthreads();
    const double isg = FINAL ? coef[0] : 0.0;
    const double h = FINAL ? coef[1] : 0.0;
    const double iom = FINAL ? coef[2] : 0.0;
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double qv[NC > 0 ? NC : 1];
#pragma unroll
        for (int k = 0; k < NC; ++k) qv[k] = Q[(int64_t)(c0 + k) * ld + i];
        double ci = c[i], wi = w[i];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            ci -= cs[k] * qv[k];
            wi -= cp[k] * qv[k];
        }
        if (FINAL) {
            const double qj = ci * isg;
            const double cn = (wi - h * qj) * iom;
            c[i] = qj;
            w[i] = cn;
            acc[0] += cn * cn;
        } else {
            c[i] = ci;
            w[i] = wi;
        }
    }
    if (FINAL) block_sums<1>(acc, 1, partial);
}

__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ partial,
                                                double *__restrict__ out,
                                                const double *__restrict__ add, int k, int sqrt_last,
                                                int nparts)
{
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

hipError_t launch_reduce(const double *partial, int k, double *out, const double *add,
                         bool sqrt_last, hipStream_t st, int nparts)
{
    hipLaunchKernelGGL(k_reduce, dim3(k), dim3(256), 0, st, partial, out, add, k, sqrt_last ? 1 : 0,
                       nparts);
    return hipGetLastError();
}

#define FE_NC_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) \
    X(14) X(15) X(16) X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) \
    X(29) X(30) X(31) X(32)

// Dot pass over the basis columns c0 .. c0 + nc - 1 (0 <= nc <= DGS_GROUP;
// nc = 0 only for the first group of a step with no final basis vector yet).
static hipError_t dgs_dots_group(int nc, bool w, bool first, const double *V, int64_t ld, int J,
                                 int c0, int64_t n, double *partial, hipStream_t st)
{
    const dim3 g(red_blocks(n)), b(RED_THREADS);
#define FE_DD(NC, W, F) hipLaunchKernelGGL((k_dgs_dots<NC, W, F>), g, b, 0, st, V, ld, J, c0, n, partial)
    if (nc == 0) {
        if (!first) return hipErrorInvalidValue;
        if (w)
            FE_DD(0, true, true);
        else
            FE_DD(0, false, true);
        return hipGetLastError();
    }
    switch (nc) {
#define FE_DC(K)                                     \
    case K:                                          \
        if (first && w)                              \
            FE_DD(K, true, true);                    \
        else if (first)                              \
            FE_DD(K, false, true);                   \
        else if (w)                                  \
            FE_DD(K, true, false);                   \
        else                                         \
            FE_DD(K, false, false);                  \
        break;
        FE_NC_CASES(FE_DC)
#undef FE_DC
    default:
        return hipErrorInvalidValue;
    }
#undef FE_DD
    return hipGetLastError();
}

static hipError_t dgs_dots(bool w, const double *V, int64_t ld, int J, int64_t n, double *partial,
                           hipStream_t st)
{
    for (int c0 = 0;; c0 += DGS_GROUP) {
        const int nc = std::min(DGS_GROUP, J - c0);
        const hipError_t e = dgs_dots_group(nc, w, c0 == 0, V, ld, J, c0, n, partial, st);
        if (e != hipSuccess) return e;
        if (c0 + DGS_GROUP >= J) return hipSuccess;
    }
}

hipError_t launch_dgs_step(double *V, int64_t ld, int J, int64_t n, double *hb, double *partial,
                           hipStream_t st)
{
    if (J < 0 || J > 63) return hipErrorInvalidValue;
    const int np = red_blocks(n);
    hipError_t e;
    if ((e = dgs_dots(true, V, ld, J, n, partial, st)) != hipSuccess) return e;
    if ((e = launch_reduce(partial, 2 * J + 3, hb, nullptr, false, st, np)) != hipSuccess) return e;
    double *c = V + (int64_t)J * ld, *w = V + (int64_t)(J + 1) * ld;
    const dim3 g(np), b(RED_THREADS);
    int c0 = 0;
    if (J > DGS_GROUP) {  // the first DGS_GROUP columns in place, the rest with the final step
        hipLaunchKernelGGL((k_dgs_update<DGS_GROUP, false>), g, b, 0, st, (const double *)V, c, w, ld,
                           J, 0, n, hb, partial);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        c0 = DGS_GROUP;
    }
    switch (J - c0) {
#define FE_UF(K)                                                                              \
    case K:                                                                                   \
        hipLaunchKernelGGL((k_dgs_update<K, true>), g, b, 0, st, (const double *)V, c, w, ld, J, \
                           c0, n, hb, partial);                                              \
        break;
        FE_UF(0)
        FE_NC_CASES(FE_UF)
#undef FE_UF
    default:
        return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_reduce(partial, 1, hb + 2 * J + 8, nullptr, false, st, np);
}

hipError_t launch_dgs_final(const double *V, int64_t ld, int J, int64_t n, double *hb,
                            double *partial, hipStream_t st)
{
    if (J < 1 || J > 64) return hipErrorInvalidValue;
    hipError_t e;
    if ((e = dgs_dots(false, V, ld, J, n, partial, st)) != hipSuccess) return e;
    return launch_reduce(partial, J + 1, hb, nullptr, false, st, red_blocks(n));
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
