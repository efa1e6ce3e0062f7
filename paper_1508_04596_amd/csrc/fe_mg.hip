// Grid-transfer, smoothing and small-level kernels of the geometric multigrid
// preconditioner (Sec. "Solving the linear systems": flexible GMRES with a
// geometric multigrid preconditioner; here the coarse operators are
// rediscretised on the coarse grid instead of formed by Galerkin projection,
// since the fine operator is never assembled).  Small levels apply their
// rediscretised operator as an assembled 27-point block stencil, and the
// coarsest level through an explicit inverse formed from its band LU factors.
//
// Coarse grids halve the element count in every direction; coarse node
// (I,J,K) coincides with fine node (2I,2J,2K).  Prolongation is trilinear
// interpolation, restriction its transpose (weights 1, 1/2, 1/4, 1/8).
#include "fe_batch.h"
#include "fe_internal.h"

namespace fe {
namespace {

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// coarse element = mean of its children (design and source): 8, or fewer where
// an odd fine grid leaves the last coarse layer half outside it
__global__ void k_coarsen_elem(int ncx, int ncy, int ncz, int nfx, int nfy, int nfz,
                               const double *__restrict__ f, double *__restrict__ c)
{
    const int64_t nc = (int64_t)ncx * ncy * ncz;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nc) return;
    const int I = (int)(e % ncx);
    const int64_t r = e / ncx;
    const int J = (int)(r % ncy), K = (int)(r / ncy);
    double s = 0.0;
    int cnt = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int i = 2 * I + dx, j = 2 * J + dy, k = 2 * K + dz;
                if (i >= nfx || j >= nfy || k >= nfz) continue;
                s += f[i + (int64_t)nfx * (j + (int64_t)nfy * k)];
                ++cnt;
            }
    c[e] = s / cnt;  // cnt is 1, 2, 4 or 8: the division is exact scaling
}

// coarse node values taken from the coincident fine node (NV values per node)
// (a coarse node past the end of an odd fine grid takes the fine boundary node)
template <typename Tf, typename Tc, int NV>
__global__ void k_inject(int ncx, int ncy, int ncz, int nfx, int nfy, int nfz,
                         const Tf *__restrict__ f, Tc *__restrict__ c)
{
    const int64_t nn = (int64_t)(ncx + 1) * (ncy + 1) * (ncz + 1);
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int I = (int)(n % (ncx + 1));
    const int64_t r = n / (ncx + 1);
    const int J = (int)(r % (ncy + 1)), K = (int)(r / (ncy + 1));
    const int i = min(2 * I, nfx), j = min(2 * J, nfy), k = min(2 * K, nfz);
    const int64_t fn = i + (int64_t)(nfx + 1) * (j + (int64_t)(nfy + 1) * k);
#pragma unroll
    for (int q = 0; q < NV; ++q) c[NV * n + q] = (Tc)f[NV * fn + q];
}

// b_c = R (b - t) on unprescribed coarse DOFs, 0 on prescribed ones; one
// thread per coarse DOF.  The 27 fine neighbours are unrolled with clamped
// addresses and a select for those outside the grid, so that their loads are
// in flight together (a loop that skips them issues one neighbour at a time);
// the sum keeps the dz, dy, dx order.
template <typename T>
__device__ __forceinline__ void restrict_dofs(int ncx, int ncy, int ncz, int nfx, int nfy, int nfz,
                                              const T *__restrict__ b, const T *__restrict__ t,
                                              const uint8_t *__restrict__ cmask, T *__restrict__ bc,
                                              unsigned blk)
{
    const int64_t nn = (int64_t)(ncx + 1) * (ncy + 1) * (ncz + 1);
    const int64_t q = (int64_t)blk * blockDim.x + threadIdx.x;
    if (q >= NF * nn) return;
    const int64_t n = q / NF;
    const int f = (int)(q - NF * n);
    const int I = (int)(n % (ncx + 1));
    const int64_t r = n / (ncx + 1);
    const int J = (int)(r % (ncy + 1)), K = (int)(r / (ncy + 1));
    T acc = T(0);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
        const int k = 2 * K + dz;
        const bool inz = k >= 0 && k <= nfz;
        const int kc = k < 0 ? 0 : (k > nfz ? nfz : k);
        const T wz = dz == 0 ? T(1) : T(0.5);
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const int j = 2 * J + dy;
            const bool iny = j >= 0 && j <= nfy;
            const int jc = j < 0 ? 0 : (j > nfy ? nfy : j);
            const T wy = dy == 0 ? T(1) : T(0.5);
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int i = 2 * I + dx;
                const bool in = inz && iny && i >= 0 && i <= nfx;
                const int ic = i < 0 ? 0 : (i > nfx ? nfx : i);
                const T w = (dx == 0 ? T(1) : T(0.5)) * wy * wz;
                const int64_t fn = ic + (int64_t)(nfx + 1) * (jc + (int64_t)(nfy + 1) * kc);
                const T v = w * (b[NF * fn + f] - (t ? t[NF * fn + f] : T(0)));
                acc += in ? v : T(0);
            }
        }
    }
    bc[q] = ((cmask[n] >> f) & 1) ? T(0) : acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_restrict(int ncx, int ncy, int ncz, int nfx, int nfy,
                                                  int nfz, const T *__restrict__ b,
                                                  const T *__restrict__ t,
                                                  const uint8_t *__restrict__ cmask,
                                                  T *__restrict__ bc)
{
    restrict_dofs<T>(ncx, ncy, ncz, nfx, nfy, nfz, b, t, cmask, bc, blockIdx.x);
}

// The restriction above fused with the first smoothing sweep of the coarse
// level, which starts from x_c = 0: x_c = omega D_c^{-1} b_c (D_c^{-T} when
// TR).  A workgroup of 255 threads covers the 5 DOFs of 51 coarse nodes; b_c
// of a node reaches its other four threads through LDS.  Both results are
// bitwise those of k_restrict followed by k_smooth (same terms, same order).
template <typename T, bool TR>
__device__ __forceinline__ void restrict_smooth_nodes(int ncx, int ncy, int ncz, int nfx, int nfy,
                                                      int nfz, const T *__restrict__ b,
                                                      const T *__restrict__ t,
                                                      const uint8_t *__restrict__ cmask,
                                                      T *__restrict__ bc, const T *__restrict__ Dc,
                                                      T *__restrict__ xc, T omega, unsigned blk)
{
    __shared__ T sb[255];
    const int64_t nn = (int64_t)(ncx + 1) * (ncy + 1) * (ncz + 1);
    const int lq = (int)threadIdx.x;
    const int ln = lq / NF, f = lq - NF * ln;
    const int64_t n = (int64_t)blk * 51 + ln;
    const bool valid = n < nn;
    T val = T(0);
    if (valid) {
        const int I = (int)(n % (ncx + 1));
        const int64_t r = n / (ncx + 1);
        const int J = (int)(r % (ncy + 1)), K = (int)(r / (ncy + 1));
        T acc = T(0);
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz) {
            const int k = 2 * K + dz;
            const bool inz = k >= 0 && k <= nfz;
            const int kc = k < 0 ? 0 : (k > nfz ? nfz : k);
            const T wz = dz == 0 ? T(1) : T(0.5);
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const int j = 2 * J + dy;
                const bool iny = j >= 0 && j <= nfy;
                const int jc = j < 0 ? 0 : (j > nfy ? nfy : j);
                const T wy = dy == 0 ? T(1) : T(0.5);
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int i = 2 * I + dx;
                    const bool in = inz && iny && i >= 0 && i <= nfx;
                    const int ic = i < 0 ? 0 : (i > nfx ? nfx : i);
                    const T w = (dx == 0 ? T(1) : T(0.5)) * wy * wz;
                    const int64_t fn = ic + (int64_t)(nfx + 1) * (jc + (int64_t)(nfy + 1) * kc);
                    const T v = w * (b[NF * fn + f] - (t ? t[NF * fn + f] : T(0)));
                    acc += in ? v : T(0);
                }
            }
        }
        val = ((cmask[n] >> f) & 1) ? T(0) : acc;
        bc[NF * n + f] = val;
    }
    sb[lq] = val;
    __syncthreads();
    if (!valid) return;
    const T *Dn = Dc + n * 25;
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < NF; ++c) acc += (TR ? Dn[c * NF + f] : Dn[f * NF + c]) * sb[NF * ln + c];
    xc[NF * n + f] = omega * acc;
}

template <typename T, bool TR>
__global__ __launch_bounds__(255) void k_restrict_smooth(int ncx, int ncy, int ncz, int nfx,
                                                         int nfy, int nfz, const T *__restrict__ b,
                                                         const T *__restrict__ t,
                                                         const uint8_t *__restrict__ cmask,
                                                         T *__restrict__ bc,
                                                         const T *__restrict__ Dc,
                                                         T *__restrict__ xc, T omega)
{
    restrict_smooth_nodes<T, TR>(ncx, ncy, ncz, nfx, nfy, nfz, b, t, cmask, bc, Dc, xc, omega,
                                 blockIdx.x);
}

// x += P xc on unprescribed fine DOFs (trilinear interpolation); one thread
// per fine DOF.  The up to 8 coarse parents are unrolled (along an even index
// the parent repeats with its term dropped) so that their loads issue together.
template <typename T>
__device__ __forceinline__ void prolong_add_dofs(int nfx, int nfy, int nfz, int ncx, int ncy,
                                                 const T *__restrict__ xc,
                                                 const uint8_t *__restrict__ fmask,
                                                 T *__restrict__ x, unsigned blk)
{
    const int64_t nn = (int64_t)(nfx + 1) * (nfy + 1) * (nfz + 1);
    const int64_t q = (int64_t)blk * blockDim.x + threadIdx.x;
    if (q >= NF * nn) return;
    const int64_t n = q / NF;
    const int f = (int)(q - NF * n);
    const int i = (int)(n % (nfx + 1));
    const int64_t r = n / (nfx + 1);
    const int j = (int)(r % (nfy + 1)), k = (int)(r / (nfy + 1));
    const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
    const int oi = i & 1, oj = j & 1, ok = k & 1;  // a second parent along odd directions
    const T wi = oi ? T(0.5) : T(1), wj = oj ? T(0.5) : T(1), wk = ok ? T(0.5) : T(1);
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int bq = 0; bq < 2; ++bq)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const bool use = (c <= ok) && (bq <= oj) && (a <= oi);
                const int64_t cn = (I0 + a * oi) + (int64_t)(ncx + 1) * ((J0 + bq * oj) + (int64_t)(ncy + 1) * (K0 + c * ok));
                const T v = xc[NF * cn + f];
                acc += use ? v : T(0);
            }
    // branch-free: the load of x is issued with the mask load instead of after it
    const int m = fmask[n];
    const T xq = x[q];
    x[q] = ((m >> f) & 1) ? xq : xq + wi * wj * wk * acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong_add(int nfx, int nfy, int nfz, int ncx, int ncy,
                                                     const T *__restrict__ xc,
                                                     const uint8_t *__restrict__ fmask, T *__restrict__ x)
{
    prolong_add_dofs<T>(nfx, nfy, nfz, ncx, ncy, xc, fmask, x, blockIdx.x);
}

// out = A v (A^T v when TR) for an assembled 27-point block stencil
// S[((d 5 + g) 5 + f) nn + N] (entry (N g, N + offset(d) f)).  A block of 9
// waves computes 64 output DOFs (node index fastest, so that stencil loads
// coalesce): wave p sums the three offsets d = 3p .. 3p + 2 over the five
// fields, all 30 loads of a lane in flight together, and the nine partials are
// added in wave order through LDS.  Row (N g) of A^T is column (N g) of A: entry
// (M f, N g) sits in row M at the opposite offset 26 - d.  Neighbours outside
// the grid load a clamped node and drop the term.
template <typename T, bool TR>
__device__ __forceinline__ void stencil_apply_dofs(int nx, int ny, int nz, const T *__restrict__ S,
                                                   const T *__restrict__ v, T *__restrict__ out,
                                                   unsigned blk)
{
    __shared__ T part[9][64];
    const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    const int lane = threadIdx.x & 63, p = threadIdx.x >> 6;
    const int64_t q = (int64_t)blk * 64 + lane;
    const bool live = q < NF * nn;
    const int g = live ? (int)(q / nn) : 0;
    const int64_t N = live ? q - (int64_t)g * nn : 0;
    const int I = (int)(N % (nx + 1));
    const int64_t r = N / (nx + 1);
    const int J = (int)(r % (ny + 1)), K = (int)(r / (ny + 1));
    const int j = J + p % 3 - 1, k = K + p / 3 - 1;
    const bool injk = j >= 0 && j <= ny && k >= 0 && k <= nz;
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int d = 3 * p + c, i = I + c - 1;
        const bool in = live && injk && i >= 0 && i <= nx;
        const int64_t M = in ? i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k) : N;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T a = TR ? S[((26 - d) * 25 + f * NF + g) * nn + M] : S[(d * 25 + g * NF + f) * nn + N];
            const T t = a * v[NF * M + f];
            acc += in ? t : T(0);
        }
    }
    part[p][lane] = acc;
    __syncthreads();
    if (p == 0 && live) {
        T sum = part[0][lane];
#pragma unroll
        for (int w = 1; w < 9; ++w) sum += part[w][lane];
        out[NF * N + g] = sum;
    }
}

template <typename T, bool TR>
__global__ __launch_bounds__(576) void k_stencil_apply(int nx, int ny, int nz, const T *__restrict__ S,
                                                       const T *__restrict__ v, T *__restrict__ out)
{
    stencil_apply_dofs<T, TR>(nx, ny, nz, S, v, out, blockIdx.x);
}

// One damped block-Jacobi sweep on an assembled level in one kernel:
// x_out = x_in + omega D^{-1} (b - A x_in) (A^T and D^{-T} when TR) for
// STENCIL_SMOOTH_NODES (32) nodes per workgroup of 9 waves.  Wave p sums the
// offsets d = 3p .. 3p + 2; lanes 0-31 of a wave hold row fields 0-2 of the 32
// nodes, lanes 32-63 row fields 3-4, so a lane issues at most 45 stencil loads
// (with 64 nodes and all five rows per lane it was 75, and the small levels
// this sweep serves left the GPU short of waves).  Each row's partial is the
// same sum as before, the nine partials of a row are added in wave order (as
// in k_stencil_apply), and the node's update is that of k_smooth, so x_out is
// bitwise the result of the two-kernel sweep.  x_out must not alias x_in
// (other workgroups read x_in at their neighbours).
template <typename T, bool TR>
__device__ __forceinline__ void stencil_smooth_nodes(int nx, int ny, int nz, const T *__restrict__ S,
                                                     const T *__restrict__ D,
                                                     const T *__restrict__ b,
                                                     const T *__restrict__ xin,
                                                     T *__restrict__ xout, T omega, unsigned blk)
{
    constexpr int SN = STENCIL_SMOOTH_NODES;
    __shared__ T part[9][NF][SN];
    __shared__ T sD[SN * 25];
    const int64_t nn = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    const int lane = threadIdx.x & 63, p = threadIdx.x >> 6;
    const int ln = lane & (SN - 1), half = lane >> 5;  // node of the block, row half
    const int g0 = half ? 3 : 0, ng = half ? NF - 3 : 3;
    const int64_t n0 = (int64_t)blk * SN;
    // the workgroup's nodal blocks, coalesced (entries past nn repeat the last)
    {
        const int64_t left = nn - n0;
        const int cnt = (int)(left < SN ? left : SN) * 25;
        const T *src = D + n0 * 25;
#pragma unroll
        for (int k = 0; k < (SN * 25 + 575) / 576; ++k) {
            const int q = (int)threadIdx.x + 576 * k;
            if (q < SN * 25) sD[q] = src[q < cnt ? q : cnt - 1];
        }
    }
    const int64_t N = n0 + ln;
    const bool live = N < nn;
    const int64_t Nc = live ? N : nn - 1;
    const int I = (int)(Nc % (nx + 1));
    const int64_t r = Nc / (nx + 1);
    const int J = (int)(r % (ny + 1)), K = (int)(r / (ny + 1));
    const int j = J + p % 3 - 1, k = K + p / 3 - 1;
    const bool injk = j >= 0 && j <= ny && k >= 0 && k <= nz;
    T xm[3][NF];
    int64_t Mc[3];
    bool inc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int i = I + c - 1;
        inc[c] = live && injk && i >= 0 && i <= nx;
        Mc[c] = inc[c] ? i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k) : Nc;
#pragma unroll
        for (int f = 0; f < NF; ++f) xm[c][f] = xin[NF * Mc[c] + f];
    }
#pragma unroll
    for (int gg = 0; gg < 3; ++gg) {
        if (gg < ng) {
            const int g = g0 + gg;
            T acc = T(0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int d = 3 * p + c;
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const T a = TR ? S[((26 - d) * 25 + f * NF + g) * nn + Mc[c]]
                                   : S[(d * 25 + g * NF + f) * nn + Nc];
                    const T t = a * xm[c][f];
                    acc += inc[c] ? t : T(0);
                }
            }
            part[p][g][ln] = acc;
        }
    }
    __syncthreads();
    if (p == 0 && half == 0 && live) {
        const T *Dn = sD + ln * 25;
        T rr[NF];
#pragma unroll
        for (int g = 0; g < NF; ++g) {
            T sum = part[0][g][ln];
#pragma unroll
            for (int w = 1; w < 9; ++w) sum += part[w][g][ln];
            rr[g] = b[NF * N + g] - sum;
        }
#pragma unroll
        for (int a = 0; a < NF; ++a) {
            T acc = T(0);
#pragma unroll
            for (int c = 0; c < NF; ++c) acc += (TR ? Dn[c * NF + a] : Dn[a * NF + c]) * rr[c];
            xout[NF * N + a] = xin[NF * N + a] + omega * acc;
        }
    }
}

template <typename T, bool TR>
__global__ __launch_bounds__(576) void k_stencil_smooth(int nx, int ny, int nz, const T *__restrict__ S,
                                                        const T *__restrict__ D,
                                                        const T *__restrict__ b,
                                                        const T *__restrict__ xin,
                                                        T *__restrict__ xout, T omega)
{
    stencil_smooth_nodes<T, TR>(nx, ny, nz, S, D, b, xin, xout, omega, blockIdx.x);
}

// The first sweep from x = 0 of a mixed-precision V-cycle, reading the FP64
// Krylov vector: b32 = (float) v and x = omega D^{-1} b32 (D^{-T} when TR) per
// node -- bitwise k_cast followed by k_smooth<float, TR, false>.
template <bool TR>
__device__ __forceinline__ void smooth0_cast_nodes(const float *__restrict__ D,
                                                   const double *__restrict__ v,
                                                   float *__restrict__ b32, float *__restrict__ x,
                                                   int64_t nn, float omega, unsigned blk)
{
    __shared__ float sD[256 * 25];
    const int64_t n0 = (int64_t)blk * 256;
    const float *Dn = stage_blocks256(D, n0, nn, sD);
    const int64_t n = n0 + threadIdx.x;
    if (n >= nn) return;
    float r[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        r[f] = (float)v[NF * n + f];
        b32[NF * n + f] = r[f];
    }
#pragma unroll
    for (int a = 0; a < NF; ++a) {
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < NF; ++c) acc += (TR ? Dn[c * NF + a] : Dn[a * NF + c]) * r[c];
        x[NF * n + a] = omega * acc;
    }
}

template <bool TR>
__global__ __launch_bounds__(256) void k_smooth0_cast(const float *__restrict__ D,
                                                      const double *__restrict__ v,
                                                      float *__restrict__ b32, float *__restrict__ x,
                                                      int64_t nn, float omega)
{
    smooth0_cast_nodes<TR>(D, v, b32, x, nn, omega, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(const T *__restrict__ a, T *__restrict__ b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// ---- coarsest level: explicit inverse from the band LU factors ---------------

// Factors of P A = L U as the host factorisation leaves them (partial pivoting
// interleaved with the elimination): column k of L holds kl multipliers
// Lc[k kl + q] (row k + 1 + q); column k of U above the diagonal holds
// Uc[k w + t] = U(k - w + t, k), w = kl + ku; Ud[k] = U(k, k); row k was
// swapped with row piv[k] >= k before column k was eliminated.
//
// A block of CI_T threads computes two columns j0, j0 + 1 of X = A^{-1} by the
// same forward and back substitution as a single solve, applied to unit
// vectors held in LDS (Y[i 2 + r], row i of right-hand side r).  Each step is
// one multiply-subtract of a factor column followed by a barrier; the factor
// column, pivot and diagonal of step k + CI_D are loaded at step k into one of
// CI_D register sets (the step loop is unrolled CI_D times so the sets stay in
// registers) and the barrier waits for LDS only, so these loads stay in flight
// across CI_D steps.  With LONG, columns longer than the register sets load
// the rest directly.  Forward steps before j0 - kl only move zeros and are
// skipped.  The back substitution finishes row k at step k and writes it to X
// (by columns: X[j n + i] = (A^{-1})_ij).
constexpr int CI_T = 256;
constexpr int CI_PFF = 2;  // forward: up to 2 CI_T entries (kl <= 256) from registers
constexpr int CI_PFB = 4;  // back: up to 4 CI_T entries (kl + ku <= 512) from registers
constexpr int CI_D = 8;

// A zero the compiler cannot see through: indexing with it turns a uniform
// load into a vector load, which the step loop waits for by vmcnt together
// with the factor columns (a scalar load would be waited for by every LDS
// access of the following steps).
__device__ __forceinline__ int ci_vzero()
{
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    return z;
}

// Barrier for LDS only: the fences are restricted to the local address space,
// so global loads in flight are not waited for.
__device__ __forceinline__ void ci_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

struct CiFwd {
    double v[CI_PFF];
    int p;
};
struct CiBack {
    double v[CI_PFB];
    double d;
};

__device__ __forceinline__ void ci_load_fwd(int k, int n, int kl, const double *__restrict__ Lc,
                                            const int *__restrict__ piv, int tid, CiFwd &c)
{
    // branch-free: entries past the column load its first entry and are zeroed
    const bool live = k < n;
    const int cnt = live ? (min(n - 1, k + kl) - k) * 2 : 0;
    const double *col = Lc + (int64_t)(live ? k : 0) * kl;
    const int pl = piv[(live ? k : 0) + ci_vzero()];
    c.p = live ? pl : 0;
#pragma unroll
    for (int m = 0; m < CI_PFF; ++m) {
        const int idx = tid + CI_T * m;
        const double t = col[idx < cnt ? idx >> 1 : 0];
        c.v[m] = idx < cnt ? t : 0.0;
    }
}

__device__ __forceinline__ void ci_load_back(int k, int w, const double *__restrict__ Uc,
                                             const double *__restrict__ Ud, int tid, CiBack &c)
{
    const bool live = k >= 0;
    const int rows = live ? min(w, k) : 0, cnt = rows * 2;
    const double *col = cnt > 0 ? Uc + (int64_t)k * w + (w - rows) : Uc;
    const double dl = Ud[(live ? k : 0) + ci_vzero()];
    c.d = live ? dl : 1.0;
#pragma unroll
    for (int m = 0; m < CI_PFB; ++m) {
        const int idx = tid + CI_T * m;
        const double t = col[idx < cnt ? idx >> 1 : 0];
        c.v[m] = idx < cnt ? t : 0.0;
    }
}

template <bool LONG>
__global__ __launch_bounds__(CI_T) void k_coarse_inverse(int n, int kl, int w, const double *__restrict__ Lc,
                                                         const double *__restrict__ Uc,
                                                         const double *__restrict__ Ud,
                                                         const int *__restrict__ piv,
                                                         double *__restrict__ X)
{
    extern __shared__ double Y[];  // 2 n entries
    const int tid = threadIdx.x;
    const int j0 = 2 * blockIdx.x;
    const bool two = j0 + 1 < n;
    for (int idx = tid; idx < 2 * n; idx += CI_T) Y[idx] = ((idx >> 1) == j0 + (idx & 1)) ? 1.0 : 0.0;
    ci_sync();
    // forward: swaps and the multipliers of L
    const int k0 = max(0, j0 - kl);
    {
        CiFwd F[CI_D];
#pragma unroll
        for (int u = 0; u < CI_D; ++u) ci_load_fwd(k0 + u, n, kl, Lc, piv, tid, F[u]);
        for (int kb = k0; kb < n; kb += CI_D) {
#pragma unroll
            for (int u = 0; u < CI_D; ++u) {
                const int k = kb + u;
                if (k >= n) break;
                const int p = __builtin_amdgcn_readfirstlane(F[u].p);
                if (p != k) {
                    if (tid < 2) {
                        const double t = Y[2 * k + tid];
                        Y[2 * k + tid] = Y[2 * p + tid];
                        Y[2 * p + tid] = t;
                    }
                    ci_sync();
                }
                const double y0 = Y[2 * k], y1 = Y[2 * k + 1];
                const int cnt = (min(n - 1, k + kl) - k) * 2;
                double *yk = Y + 2 * (k + 1);
#pragma unroll
                for (int m = 0; m < CI_PFF; ++m) {
                    const int idx = tid + CI_T * m;
                    if (idx < cnt) yk[idx] -= F[u].v[m] * ((idx & 1) ? y1 : y0);
                }
                if (LONG) {
                    const double *lk = Lc + (int64_t)k * kl;
                    for (int idx = tid + CI_T * CI_PFF; idx < cnt; idx += CI_T)
                        yk[idx] -= lk[idx >> 1] * ((idx & 1) ? y1 : y0);
                }
                ci_load_fwd(k + CI_D, n, kl, Lc, piv, tid, F[u]);
                ci_sync();
            }
        }
    }
    // back substitution with U, by columns: step k updates rows max(0, k - w) .. k - 1
    {
        CiBack B[CI_D];
#pragma unroll
        for (int u = 0; u < CI_D; ++u) ci_load_back(n - 1 - u, w, Uc, Ud, tid, B[u]);
        for (int kb = n - 1; kb >= 0; kb -= CI_D) {
#pragma unroll
            for (int u = 0; u < CI_D; ++u) {
                const int k = kb - u;
                if (k < 0) break;
                const double x0 = Y[2 * k] / B[u].d, x1 = Y[2 * k + 1] / B[u].d;
                const int rows = min(w, k), cnt = 2 * rows;
                double *yr = Y + 2 * (k - rows);
#pragma unroll
                for (int m = 0; m < CI_PFB; ++m) {
                    const int idx = tid + CI_T * m;
                    if (idx < cnt) yr[idx] -= B[u].v[m] * ((idx & 1) ? x1 : x0);
                }
                if (LONG) {
                    const double *uk = Uc + (int64_t)k * w + (w - rows);
                    for (int idx = tid + CI_T * CI_PFB; idx < cnt; idx += CI_T)
                        yr[idx] -= uk[idx >> 1] * ((idx & 1) ? x1 : x0);
                }
                if (tid == 0) X[(int64_t)j0 * n + k] = x0;
                if (tid == 1 && two) X[(int64_t)(j0 + 1) * n + k] = x1;
                ci_load_back(k - CI_D, w, Uc, Ud, tid, B[u]);
                ci_sync();
            }
        }
    }
}

// x = A^{-1} b (A^{-T} b when TR) on the coarsest level in two passes, FP64
// accumulation in a fixed order.  A is the matrix restricted to the n free DOFs
// (fidx: free -> full index); prescribed DOFs have identity rows and zero
// columns in the full matrix, so their x is b.  Pass 1: block (rb, cb)
// multiplies the 64 x 64 tile of rows rb and columns cb of the condensed
// inverse by the matching 64 free entries of b and writes the 64 row partials
// to P[cb n + i]; pass 2 adds the partials of each row in chunk order and
// scatters to the full vector.  X is stored by columns (X[j n + i] = (A^{-1})_ij), so
// for A^{-1} the tile is read along its rows' index i (wave q takes columns
// q, q + 4, ...), for A^{-T} along j (wave q takes rows q, q + 4, ...; a row's 64
// products are summed through LDS).
constexpr int CA_B = 64;

template <typename T, bool TR>
__device__ __forceinline__ void coarse_apply_tile(int n, const double *__restrict__ X,
                                                  const int *__restrict__ fidx,
                                                  const T *__restrict__ b, double *__restrict__ P,
                                                  unsigned bx, unsigned by)
{
    __shared__ double tile[4][CA_B + 1];
    __shared__ double prod[CA_B][CA_B + 1];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int i0 = bx * CA_B, j0 = by * CA_B;
    if (!TR) {
        const int i = i0 + lane;
        const int ic = i < n ? i : n - 1;
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < CA_B / 4; ++m) {
            const int j = j0 + q + 4 * m;
            const int jc = j < n ? j : n - 1;
            const double t = X[(int64_t)jc * n + ic] * (double)b[fidx[jc]];
            acc += j < n ? t : 0.0;
        }
        tile[q][lane] = acc;
        __syncthreads();
        if (q == 0 && i < n)
            P[(int64_t)by * n + i] = ((tile[0][lane] + tile[1][lane]) + tile[2][lane]) + tile[3][lane];
    } else {
        const int j = j0 + lane;
        const int jc = j < n ? j : n - 1;
        const double bj = j < n ? (double)b[fidx[jc]] : 0.0;
#pragma unroll
        for (int m = 0; m < CA_B / 4; ++m) {
            const int r = q + 4 * m;
            const int i = i0 + r;
            const int ic = i < n ? i : n - 1;
            prod[r][lane] = X[(int64_t)ic * n + jc] * bj;
        }
        __syncthreads();
        if (threadIdx.x < CA_B) {
            const int i = i0 + threadIdx.x;
            double acc = 0.0;
            for (int l = 0; l < CA_B; ++l) acc += prod[threadIdx.x][l];
            if (i < n) P[(int64_t)by * n + i] = acc;
        }
    }
}

template <typename T, bool TR>
__global__ __launch_bounds__(256) void k_coarse_apply_part(int n, const double *__restrict__ X,
                                                           const int *__restrict__ fidx,
                                                           const T *__restrict__ b, double *__restrict__ P)
{
    coarse_apply_tile<T, TR>(n, X, fidx, b, P, blockIdx.x, blockIdx.y);
}

// Pass 2 over the full vector (nfull DOFs; pos: full -> free index, -1 when prescribed).
template <typename T>
__device__ __forceinline__ void coarse_apply_rows(int nfull, int n, int nc, const int *__restrict__ pos,
                                                  const double *__restrict__ P,
                                                  const T *__restrict__ b, T *__restrict__ x,
                                                  unsigned blk)
{
    const int i = blk * blockDim.x + threadIdx.x;
    if (i >= nfull) return;
    const int r = pos[i];
    if (r < 0) {
        x[i] = b[i];
        return;
    }
    double acc = 0.0;
#pragma unroll 8
    for (int c = 0; c < nc; ++c) acc += P[(int64_t)c * n + r];
    x[i] = (T)acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_coarse_apply_sum(int nfull, int n, int nc, const int *__restrict__ pos,
                                                          const double *__restrict__ P,
                                                          const T *__restrict__ b, T *__restrict__ x)
{
    coarse_apply_rows<T>(nfull, n, nc, pos, P, b, x, blockIdx.x);
}

// Nodal diagonal blocks of an assembled level from its stencil: D[n 25 + g 5 + f]
// = S[((13 25) + g 5 + f) nn + n] (offset 13 is the node itself; prescribed rows
// and columns already carry the identity pattern the smoother expects).
__global__ __launch_bounds__(256) void k_stencil_diag(int64_t nn, const double *__restrict__ S,
                                                      double *__restrict__ D)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 25 * nn) return;
    const int64_t n = q / 25;
    const int e = (int)(q - 25 * n);
    D[q] = S[(int64_t)(13 * 25 + e) * nn + n];
}

// x (+)= omega * D^{-1} (b - t) per node (D^{-T} when TR); t may be NULL (= 0);
// ACC = false overwrites x.
// Launched with 256 threads per workgroup (the block staging assumes it).
template <typename T, bool TR, bool ACC>
__device__ __forceinline__ void smooth_nodes(const T *__restrict__ D, const T *__restrict__ b,
                                             const T *__restrict__ t, T *__restrict__ x, int64_t nn,
                                             T omega, unsigned blk)
{
    __shared__ T sD[256 * 25];
    const int64_t n0 = (int64_t)blk * 256;
    const T *Dn = stage_blocks256(D, n0, nn, sD);
    const int64_t n = n0 + threadIdx.x;
    if (n >= nn) return;
    T r[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) r[f] = b[NF * n + f] - (t ? t[NF * n + f] : T(0));
#pragma unroll
    for (int a = 0; a < NF; ++a) {
        T acc = T(0);
#pragma unroll
        for (int c = 0; c < NF; ++c) acc += (TR ? Dn[c * NF + a] : Dn[a * NF + c]) * r[c];
        if (ACC)
            x[NF * n + a] += omega * acc;
        else
            x[NF * n + a] = omega * acc;
    }
}

template <typename T, bool TR, bool ACC>
__global__ __launch_bounds__(256) void k_smooth(const T *__restrict__ D, const T *__restrict__ b,
                                                const T *__restrict__ t, T *__restrict__ x,
                                                int64_t nn, T omega)
{
    smooth_nodes<T, TR, ACC>(D, b, t, x, nn, omega, blockIdx.x);
}

// ---- batched launches: the kernels above over a table of problems -------------

template <typename T>
__global__ __launch_bounds__(576) void kb_stencil(const BStencil<T> *__restrict__ tab,
                                                  const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BStencil<T> &a = tab[e];
    stencil_apply_dofs<T, false>(a.nx, a.ny, a.nz, a.S, a.v, a.out, blockIdx.x - (unsigned)off[e]);
}

template <typename T, bool ACC>
__global__ __launch_bounds__(256) void kb_smooth(const BSmooth<T> *__restrict__ tab,
                                                 const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BSmooth<T> &a = tab[e];
    smooth_nodes<T, false, ACC>(a.D, a.b, a.t, a.x, a.nn, a.omega, blockIdx.x - (unsigned)off[e]);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_restrict(const BRestrict<T> *__restrict__ tab,
                                                   const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BRestrict<T> &a = tab[e];
    restrict_dofs<T>(a.ncx, a.ncy, a.ncz, a.nfx, a.nfy, a.nfz, a.b, a.t, a.cmask, a.bc,
                     blockIdx.x - (unsigned)off[e]);
}

template <typename T>
__global__ __launch_bounds__(255) void kb_restrict_smooth(const BRestrict<T> *__restrict__ tab,
                                                          const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BRestrict<T> &a = tab[e];
    restrict_smooth_nodes<T, false>(a.ncx, a.ncy, a.ncz, a.nfx, a.nfy, a.nfz, a.b, a.t, a.cmask,
                                    a.bc, a.Dc, a.xc, a.omega, blockIdx.x - (unsigned)off[e]);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_prolong(const BProlong<T> *__restrict__ tab,
                                                  const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BProlong<T> &a = tab[e];
    prolong_add_dofs<T>(a.nfx, a.nfy, a.nfz, a.ncx, a.ncy, a.xc, a.fmask, a.x,
                        blockIdx.x - (unsigned)off[e]);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_coarse_part(const BCoarse<T> *__restrict__ tab,
                                                      const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BCoarse<T> &a = tab[e];
    const unsigned lb = blockIdx.x - (unsigned)off[e];
    coarse_apply_tile<T, false>(a.n, a.X, a.fidx, a.b, a.P, lb % (unsigned)a.nt,
                                lb / (unsigned)a.nt);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_coarse_sum(const BCoarse<T> *__restrict__ tab,
                                                     const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BCoarse<T> &a = tab[e];
    coarse_apply_rows<T>(a.nfull, a.n, a.nt, a.pos, a.P, a.b, a.x, blockIdx.x - (unsigned)off[e]);
}

template <typename T>
__global__ __launch_bounds__(576) void kb_stencil_smooth(const BStencilSmooth<T> *__restrict__ tab,
                                                         const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BStencilSmooth<T> &a = tab[e];
    stencil_smooth_nodes<T, false>(a.nx, a.ny, a.nz, a.S, a.D, a.b, a.xin, a.xout, a.omega,
                                   blockIdx.x - (unsigned)off[e]);
}

__global__ __launch_bounds__(256) void kb_smooth0_cast(const BSmooth0Cast *__restrict__ tab,
                                                       const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BSmooth0Cast &a = tab[e];
    smooth0_cast_nodes<false>(a.D, a.v, a.b32, a.x, a.nn, a.omega, blockIdx.x - (unsigned)off[e]);
}

}  // namespace

hipError_t mg_coarsen_elem(const fe_grid &c, const fe_grid &f, const double *fv, double *cv,
                          hipStream_t st)
{
    const int64_t n = (int64_t)c.nx * c.ny * c.nz;
    hipLaunchKernelGGL(k_coarsen_elem, dim3(nblk(n)), dim3(256), 0, st, c.nx, c.ny, c.nz, f.nx, f.ny,
                       f.nz, fv, cv);
    return hipGetLastError();
}

hipError_t mg_inject_state(const fe_grid &c, const fe_grid &f, const double *fv, double *cv,
                           hipStream_t st)
{
    const int64_t n = (int64_t)(c.nx + 1) * (c.ny + 1) * (c.nz + 1);
    hipLaunchKernelGGL((k_inject<double, double, NF>), dim3(nblk(n)), dim3(256), 0, st, c.nx, c.ny,
                       c.nz, f.nx, f.ny, f.nz, fv, cv);
    return hipGetLastError();
}

hipError_t mg_inject_mask(const fe_grid &c, const fe_grid &f, const uint8_t *fv, uint8_t *cv,
                          hipStream_t st)
{
    const int64_t n = (int64_t)(c.nx + 1) * (c.ny + 1) * (c.nz + 1);
    hipLaunchKernelGGL((k_inject<uint8_t, uint8_t, 1>), dim3(nblk(n)), dim3(256), 0, st, c.nx, c.ny,
                       c.nz, f.nx, f.ny, f.nz, fv, cv);
    return hipGetLastError();
}

template <typename T>
hipError_t mg_restrict(const fe_grid &c, const fe_grid &f, const T *b, const T *t,
                       const uint8_t *cmask, T *bc, hipStream_t st)
{
    const int64_t n = (int64_t)(c.nx + 1) * (c.ny + 1) * (c.nz + 1);
    hipLaunchKernelGGL(k_restrict<T>, dim3(nblk(NF * n)), dim3(256), 0, st, c.nx, c.ny, c.nz, f.nx,
                       f.ny, f.nz, b, t, cmask, bc);
    return hipGetLastError();
}

template <typename T>
hipError_t mg_restrict_smooth(const fe_grid &c, const fe_grid &f, const T *b, const T *t,
                              const uint8_t *cmask, T *bc, const T *Dc, T *xc, T omega,
                              bool transpose, hipStream_t st)
{
    const int64_t n = (int64_t)(c.nx + 1) * (c.ny + 1) * (c.nz + 1);
    const dim3 g((unsigned)((n + 50) / 51)), bl(255);
    if (transpose)
        hipLaunchKernelGGL((k_restrict_smooth<T, true>), g, bl, 0, st, c.nx, c.ny, c.nz, f.nx, f.ny,
                           f.nz, b, t, cmask, bc, Dc, xc, omega);
    else
        hipLaunchKernelGGL((k_restrict_smooth<T, false>), g, bl, 0, st, c.nx, c.ny, c.nz, f.nx, f.ny,
                           f.nz, b, t, cmask, bc, Dc, xc, omega);
    return hipGetLastError();
}

template <typename T>
hipError_t mg_prolong_add(const fe_grid &f, const fe_grid &c, const T *xc, const uint8_t *fmask,
                          T *x, hipStream_t st)
{
    const int64_t n = (int64_t)(f.nx + 1) * (f.ny + 1) * (f.nz + 1);
    hipLaunchKernelGGL(k_prolong_add<T>, dim3(nblk(NF * n)), dim3(256), 0, st, f.nx, f.ny, f.nz,
                       c.nx, c.ny, xc, fmask, x);
    return hipGetLastError();
}

template <typename T>
hipError_t mg_stencil_apply(int nx, int ny, int nz, const T *S, const T *v, T *out, bool transpose,
                            hipStream_t st)
{
    const int64_t n = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    if (transpose)
        hipLaunchKernelGGL((k_stencil_apply<T, true>), dim3(nblk(NF * n, 64)), dim3(576), 0, st, nx, ny, nz, S, v, out);
    else
        hipLaunchKernelGGL((k_stencil_apply<T, false>), dim3(nblk(NF * n, 64)), dim3(576), 0, st, nx, ny, nz, S, v, out);
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

hipError_t mg_stencil_diag(int64_t nn, const double *S, double *D, hipStream_t st)
{
    hipLaunchKernelGGL(k_stencil_diag, dim3(nblk(25 * nn)), dim3(256), 0, st, nn, S, D);
    return hipGetLastError();
}

hipError_t mg_coarse_inverse(int n, int kl, int ku, const double *Lc, const double *Uc,
                             const double *Ud, const int *piv, double *X, hipStream_t st)
{
    const unsigned lds = (unsigned)(2 * n * sizeof(double));
    if (2 * kl <= CI_T * CI_PFF && 2 * (kl + ku) <= CI_T * CI_PFB)
        hipLaunchKernelGGL(k_coarse_inverse<false>, dim3((unsigned)((n + 1) / 2)), dim3(CI_T), lds, st,
                           n, kl, kl + ku, Lc, Uc, Ud, piv, X);
    else
        hipLaunchKernelGGL(k_coarse_inverse<true>, dim3((unsigned)((n + 1) / 2)), dim3(CI_T), lds, st,
                           n, kl, kl + ku, Lc, Uc, Ud, piv, X);
    return hipGetLastError();
}

// nfull DOFs, m of them free; X: m x m; P: work space of ceil(m / 64) * m doubles
template <typename T>
hipError_t mg_coarse_apply(int nfull, int m, const double *X, const int *fidx, const int *pos, const T *b,
                           T *x, double *P, bool transpose, hipStream_t st)
{
    const int nc = (m + CA_B - 1) / CA_B;
    const dim3 grid((unsigned)nc, (unsigned)nc);
    if (m > 0) {
        if (transpose)
            hipLaunchKernelGGL((k_coarse_apply_part<T, true>), grid, dim3(256), 0, st, m, X, fidx, b, P);
        else
            hipLaunchKernelGGL((k_coarse_apply_part<T, false>), grid, dim3(256), 0, st, m, X, fidx, b, P);
    }
    hipLaunchKernelGGL(k_coarse_apply_sum<T>, dim3((unsigned)((nfull + 255) / 256)), dim3(256), 0, st, nfull,
                       m, nc, pos, (const double *)P, b, x);
    return hipGetLastError();
}

template <typename T>
hipError_t mg_stencil_smooth(int nx, int ny, int nz, const T *S, const T *D, const T *b, const T *xin,
                             T *xout, T omega, bool transpose, hipStream_t st)
{
    const int64_t n = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    if (transpose)
        hipLaunchKernelGGL((k_stencil_smooth<T, true>), dim3(nblk(n, STENCIL_SMOOTH_NODES)),
                           dim3(576), 0, st, nx, ny, nz, S, D, b, xin, xout, omega);
    else
        hipLaunchKernelGGL((k_stencil_smooth<T, false>), dim3(nblk(n, STENCIL_SMOOTH_NODES)),
                           dim3(576), 0, st, nx, ny, nz, S, D, b, xin, xout, omega);
    return hipGetLastError();
}

hipError_t mg_smooth0_cast(const float *D, const double *v, float *b32, float *x, int64_t nn,
                           float omega, bool transpose, hipStream_t st)
{
    if (transpose)
        hipLaunchKernelGGL(k_smooth0_cast<true>, dim3(nblk(nn)), dim3(256), 0, st, D, v, b32, x, nn,
                           omega);
    else
        hipLaunchKernelGGL(k_smooth0_cast<false>, dim3(nblk(nn)), dim3(256), 0, st, D, v, b32, x,
                           nn, omega);
    return hipGetLastError();
}

template <typename T>
hipError_t mg_copy(const T *a, T *b, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy<T>, dim3(nblk(n)), dim3(256), 0, st, a, b, n);
    return hipGetLastError();
}

#define FE_MG_INST(T)                                                                          \
    template hipError_t mg_restrict<T>(const fe_grid &, const fe_grid &, const T *, const T *,      \
                                       const uint8_t *, T *,                                      \
                                       hipStream_t);                                           \
    template hipError_t mg_restrict_smooth<T>(const fe_grid &, const fe_grid &, const T *,       \
                                              const T *, const uint8_t *, T *, const T *, T *, T,  \
                                              bool, hipStream_t);                                 \
    template hipError_t mg_prolong_add<T>(const fe_grid &, const fe_grid &, const T *,           \
                                          const uint8_t *, T *,                                   \
                                          hipStream_t);                                        \
    template hipError_t mg_smooth<T>(const T *, const T *, const T *, T *, int64_t, T, bool, bool, \
                                     hipStream_t);                                             \
    template hipError_t mg_stencil_apply<T>(int, int, int, const T *, const T *, T *, bool,      \
                                            hipStream_t);                                      \
    template hipError_t mg_coarse_apply<T>(int, int, const double *, const int *, const int *,    \
                                           const T *, T *, double *, bool, hipStream_t);        \
    template hipError_t mg_stencil_smooth<T>(int, int, int, const T *, const T *, const T *,      \
                                             const T *, T *, T, bool, hipStream_t);              \
    template hipError_t mg_copy<T>(const T *, T *, int64_t, hipStream_t);
FE_MG_INST(double)
FE_MG_INST(float)
#undef FE_MG_INST

// ---- batched launchers ---------------------------------------------------------------

#define FE_BLAUNCH(NAME, KERNEL, ARGS, THREADS)                                                  \
    template <typename T>                                                                      \
    hipError_t NAME(const BLaunch &L, hipStream_t st)                                          \
    {                                                                                          \
        if (L.blocks <= 0) return hipSuccess;                                                  \
        hipLaunchKernelGGL(KERNEL, dim3((unsigned)L.blocks), dim3(THREADS), 0, st,             \
                           (const ARGS *)L.tab, L.off, L.n);                                    \
        return hipGetLastError();                                                              \
    }
FE_BLAUNCH(blaunch_stencil, kb_stencil<T>, BStencil<T>, 576)
FE_BLAUNCH(blaunch_restrict, kb_restrict<T>, BRestrict<T>, 256)
FE_BLAUNCH(blaunch_restrict_smooth, kb_restrict_smooth<T>, BRestrict<T>, 255)
FE_BLAUNCH(blaunch_prolong, kb_prolong<T>, BProlong<T>, 256)
FE_BLAUNCH(blaunch_coarse_part, kb_coarse_part<T>, BCoarse<T>, 256)
FE_BLAUNCH(blaunch_coarse_sum, kb_coarse_sum<T>, BCoarse<T>, 256)
FE_BLAUNCH(blaunch_stencil_smooth, kb_stencil_smooth<T>, BStencilSmooth<T>, 576)
#undef FE_BLAUNCH

hipError_t blaunch_smooth0_cast(const BLaunch &L, hipStream_t st)
{
    if (L.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(kb_smooth0_cast, dim3((unsigned)L.blocks), dim3(256), 0, st,
                       (const BSmooth0Cast *)L.tab, L.off, L.n);
    return hipGetLastError();
}

template <typename T, bool ACC>
hipError_t blaunch_smooth(const BLaunch &L, hipStream_t st)
{
    if (L.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((kb_smooth<T, ACC>), dim3((unsigned)L.blocks), dim3(256), 0, st,
                       (const BSmooth<T> *)L.tab, L.off, L.n);
    return hipGetLastError();
}

#define FE_BMG_INST(T)                                                                         \
    template hipError_t blaunch_stencil<T>(const BLaunch &, hipStream_t);                      \
    template hipError_t blaunch_restrict<T>(const BLaunch &, hipStream_t);                     \
    template hipError_t blaunch_restrict_smooth<T>(const BLaunch &, hipStream_t);              \
    template hipError_t blaunch_prolong<T>(const BLaunch &, hipStream_t);                      \
    template hipError_t blaunch_coarse_part<T>(const BLaunch &, hipStream_t);                  \
    template hipError_t blaunch_coarse_sum<T>(const BLaunch &, hipStream_t);                   \
    template hipError_t blaunch_stencil_smooth<T>(const BLaunch &, hipStream_t);               \
    template hipError_t blaunch_smooth<T, false>(const BLaunch &, hipStream_t);                \
    template hipError_t blaunch_smooth<T, true>(const BLaunch &, hipStream_t);
FE_BMG_INST(double)
FE_BMG_INST(float)
#undef FE_BMG_INST

}  // namespace fe
