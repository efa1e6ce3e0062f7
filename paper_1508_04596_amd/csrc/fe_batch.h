// Batched launches over a table of problems (internal).
//
// A batched launch runs one kernel over several problems at once: entry i of a
// device table holds problem i's arguments, and workgroups off[i] .. off[i+1]-1
// of the launch work on it, each with its local workgroup index
// blockIdx.x - off[i].  The element and multigrid kernels run the same device
// bodies as their one-problem launches, so a problem's result does not depend
// on which other problems share the launch, and equals that of the
// one-problem kernels.
#pragma once

#include "fe_internal.h"

namespace fe {

// One batched launch: device pointers to its argument table and to the n + 1
// workgroup offsets; blocks = off[n].
struct BLaunch {
    const void *tab = nullptr;
    const int *off = nullptr;
    int n = 0;
    int blocks = 0;
};

// Table entry that owns this workgroup (off[0] = 0 <= blockIdx.x < off[n]).
__device__ __forceinline__ int batch_entry(const int *__restrict__ off, int n)
{
    const int b = (int)blockIdx.x;
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// ---- element passes (fe_elem.hip) ------------------------------------------
// J v: the element pass writes out (and the tile-face slots), the shared-node
// pass completes out; both launches take the same table.
template <typename Tin, typename Tout>
struct BElem {
    Geo g;
    const Tin *x, *v;
    const double *gamma, *s;
    const uint8_t *nmask;
    Tout *out, *slots;
};
// One smoothing sweep x += omega D^{-1} (b - J x) of a matrix-free level
// (element pass into t and the slots, then the fused shared-node/smoothing pass).
template <typename T>
struct BElemSmooth {
    Geo g;
    const T *xs;
    T *x;
    const double *gamma, *s;
    const uint8_t *nmask;
    T *t, *slots;
    const T *D, *b;
    T omega;
};
inline int belem_blocks(const Geo &g) { return (int)n_tiles(g); }
inline int bnode_blocks(const Geo &g) { return (int)((n_nodes(g) + 255) / 256); }
template <typename Tin, typename Tout>
hipError_t blaunch_elem_jv(const BLaunch &L, hipStream_t st);
template <typename Tin, typename Tout>
hipError_t blaunch_combine_jv(const BLaunch &L, hipStream_t st);
template <typename T>
hipError_t blaunch_elem_smooth_pass(const BLaunch &L, hipStream_t st);
template <typename T>
hipError_t blaunch_combine_smooth(const BLaunch &L, hipStream_t st);

// ---- multigrid (fe_mg.hip) -------------------------------------------------
template <typename T>
struct BStencil {
    int nx, ny, nz;
    const T *S, *v;
    T *out;
};
template <typename T>
struct BSmooth {  // x (+)= omega D^{-1} (b - t); t may be NULL
    const T *D, *b, *t;
    T *x;
    int64_t nn;
    T omega;
};
template <typename T>
struct BRestrict {  // b_c = R (b - t); with Dc: also x_c = omega D_c^{-1} b_c
    int ncx, ncy, ncz, nfx, nfy, nfz;
    const T *b, *t;
    const uint8_t *cmask;
    T *bc;
    const T *Dc;
    T *xc;
    T omega;
};
template <typename T>
struct BProlong {  // x += P x_c
    int nfx, nfy, nfz, ncx, ncy;
    const T *xc;
    const uint8_t *fmask;
    T *x;
};
template <typename T>
struct BCoarse {  // x = A_c^{-1} b through the explicit inverse of the free DOFs
    int nfull, n, nt;  // DOFs, free DOFs, 64-row tiles per dimension
    const double *X;
    const int *fidx, *pos;
    const T *b;
    T *x;
    double *P;
};
template <typename T>
struct BStencilSmooth {  // x_out = x_in + omega D^{-1} (b - S x_in), x_out != x_in
    int nx, ny, nz;
    const T *S, *D, *b, *xin;
    T *xout;
    T omega;
};
struct BSmooth0Cast {  // b32 = (float) v, x = omega D^{-1} b32
    const float *D;
    const double *v;
    float *b32, *x;
    int64_t nn;
    float omega;
};
inline int bstencil_blocks(int64_t nn) { return (int)((NF * nn + 63) / 64); }
// nodes per workgroup of the one-kernel stencil sweep (k_stencil_smooth)
constexpr int STENCIL_SMOOTH_NODES = 32;
inline int bstencil_smooth_blocks(int64_t nn)
{
    return (int)((nn + STENCIL_SMOOTH_NODES - 1) / STENCIL_SMOOTH_NODES);
}
inline int bsmooth_blocks(int64_t nn) { return (int)((nn + 255) / 256); }
inline int brestrict_blocks(int64_t nn_c) { return (int)((NF * nn_c + 255) / 256); }
inline int brestrict_smooth_blocks(int64_t nn_c) { return (int)((nn_c + 50) / 51); }
inline int bprolong_blocks(int64_t nn_f) { return (int)((NF * nn_f + 255) / 256); }
inline int bcoarse_part_blocks(int n) { return n > 0 ? ((n + 63) / 64) * ((n + 63) / 64) : 0; }
inline int bcoarse_sum_blocks(int nfull) { return (nfull + 255) / 256; }
template <typename T>
hipError_t blaunch_stencil(const BLaunch &L, hipStream_t st);
template <typename T, bool ACC>
hipError_t blaunch_smooth(const BLaunch &L, hipStream_t st);
template <typename T>
hipError_t blaunch_restrict(const BLaunch &L, hipStream_t st);
template <typename T>
hipError_t blaunch_restrict_smooth(const BLaunch &L, hipStream_t st);
template <typename T>
hipError_t blaunch_prolong(const BLaunch &L, hipStream_t st);
template <typename T>
hipError_t blaunch_coarse_part(const BLaunch &L, hipStream_t st);
template <typename T>
hipError_t blaunch_coarse_sum(const BLaunch &L, hipStream_t st);
template <typename T>
hipError_t blaunch_stencil_smooth(const BLaunch &L, hipStream_t st);
hipError_t blaunch_smooth0_cast(const BLaunch &L, hipStream_t st);

// ---- vectors and reductions (fe_batch.hip) ---------------------------------
// Reductions split a problem's vector of n entries into nchunk chunks of
// 256 * ept consecutive entries (ept the smallest power of two that keeps
// nchunk <= BRED_MAX_CHUNKS, so that small vectors still spread over many
// workgroups); the chunking depends on n only, and partials are added in a
// fixed order, so a problem's sums are the same in every batch.
constexpr int BRED_MAX_CHUNKS = 1024;
constexpr int BDOT_GROUP = 8;  // basis vectors per workgroup of a multi-dot
inline void bred_chunks(int64_t n, int *nchunk, int *ept)
{
    int64_t e = 1;
    while ((n + 256 * e - 1) / (256 * e) > BRED_MAX_CHUNKS) e *= 2;
    *ept = (int)e;
    *nchunk = (int)std::max<int64_t>(1, (n + 256 * e - 1) / (256 * e));
}
struct BFill {
    double *p;
    int64_t n;
};
struct BCast {
    const double *a;
    float *b;
    int64_t n;
};
struct BWiden {  // b = (double) a
    const float *a;
    double *b;
    int64_t n;
};
struct BAxpby {  // y = a x + b y
    int64_t n;
    double a;
    const double *x;
    double b;
    double *y;
};
template <typename T>
struct BCopy {  // b = a
    const T *a;
    T *b;
    int64_t n;
};
struct BScale {  // y = x / s[0]
    int64_t n;
    const double *x, *s;
    double *y;
};
constexpr int BCOMB_MAX = 64;
template <typename Tz>
struct BComb {  // x += sum_{j<k} y_j Z_j
    const Tz *Z;
    int64_t ld;
    int k;
    int64_t n;
    double *x;
    double y[BCOMB_MAX];
};
struct BDots {  // partial[c nchunk + chunk] of <V_c, w> for c < k, and <w, w> as column k if norm
    const double *w, *V;
    int64_t ld;
    int k, norm;
    int64_t n;
    int nchunk, ept, ngrp;
    double *partial;
};
struct BScaleNorm {  // y = x / |x| with |x|^2 the sum of nchunk partials; nrm2, beta = |x|^2, |x|
    const double *partial;
    int nchunk;
    int64_t n;
    const double *x;
    double *y, *nrm2, *beta;
};
struct BReduce {  // out[c] = sum of the nchunk partials of column c < ncol (one workgroup
                  // per column); beta = sqrt(out[ncol-1])
    const double *partial;
    int ncol, nchunk;
    double *out, *beta;
};
// Delayed classical Gram-Schmidt (the one-problem FGMRES's scheme): basis
// vectors q_0 .. q_{J-1} in columns 0 .. J-1 of V, the candidate c in column J,
// the new Krylov vector w in column J + 1.
struct BDgsDots {  // partials of s_i = <q_i, c>, a = <c, c> and, if w: p_i = <q_i, w>, t = <c, w>,
                   // e = <w, w>, as columns i, J, J + 1 + i, 2J + 1, 2J + 2 (BDOT_GROUP basis
                   // columns per workgroup and chunk; the group of column 0 also takes a, t, e)
    const double *V;
    int64_t ld;
    int J, w;
    int64_t n;
    int nchunk, ept, ngrp;
    double *partial;
};
struct BDgsUpdate {  // from the reduced dot products in res: sigma, h, omega (to res[2J+3 ..
                     // 2J+5]), q_J = (c - sum s_i q_i) / sigma into column J, the next candidate
                     // (w - sum p_i q_i - h q_J) / omega into column J + 1, chunk partials of its
                     // squared norm
    double *V;
    int64_t ld;
    int J;
    int64_t n;
    int nchunk, ept;
    double *res;
    double *partial;
};
inline int belt_blocks(int64_t n) { return (int)((n + 255) / 256); }
hipError_t blaunch_fill(const BLaunch &L, hipStream_t st);
hipError_t blaunch_cast(const BLaunch &L, hipStream_t st);
hipError_t blaunch_widen(const BLaunch &L, hipStream_t st);
hipError_t blaunch_axpby(const BLaunch &L, hipStream_t st);
hipError_t blaunch_scale(const BLaunch &L, hipStream_t st);
template <typename Tz>
hipError_t blaunch_comb(const BLaunch &L, hipStream_t st);
template <typename T>
hipError_t blaunch_copy(const BLaunch &L, hipStream_t st);
hipError_t blaunch_dots(const BLaunch &L, hipStream_t st);
hipError_t blaunch_reduce(const BLaunch &L, hipStream_t st);
hipError_t blaunch_dgs_dots(const BLaunch &L, hipStream_t st);
hipError_t blaunch_dgs_update(const BLaunch &L, hipStream_t st);
hipError_t blaunch_scale_norm(const BLaunch &L, hipStream_t st);

}  // namespace fe
