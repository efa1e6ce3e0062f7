// Element kernels of the stabilised natural-convection operator on gfx950.
//
// One workgroup (256 threads, 4 wave64) owns a tile of 8x8x4 elements, one
// element per thread.  The tile's 9x9x5 node box of the state (and of the
// direction) is staged in LDS with coalesced loads, field-major so that the
// per-thread gathers of the element corners are bank-conflict free.  Each
// thread evaluates its element with the 2x2x2 Gauss rule in registers: nodal
// values are turned into the tensor-product modal basis {1, xi, eta, zeta, ...}
// by a three-pass butterfly, so the value and the three derivatives at a Gauss
// point are signed sums of eight modal coefficients; the test-function side is
// accumulated in the same modal basis and turned back into nodal rows by the
// inverse butterfly.  Element rows are summed into an LDS node accumulator in
// eight ordered sub-steps (one per element corner, so no two threads touch the
// same node within a sub-step).  Nodes whose elements all lie in the tile are
// written directly; nodes on faces shared with neighbouring tiles write their
// partial sums to per-tile slots that a second kernel adds in a fixed tile
// order.  No atomics: results are bitwise reproducible and independent of the
// launch order.
//
// Weak form, stabilisation and linearisation: Sec. "Finite element formulation"
// and Appendix "Stabilisation parameters" (tau from the convective, viscous and
// Brinkman limits; its variation with the element velocity vector enters the
// consistent Jacobian).  The viscous second derivative is left out of the
// strong residual used by SUPG/PSPG.
#include "fe_batch.h"
#include "fe_internal.h"

namespace fe {
namespace {

constexpr double QG = 0.57735026918962576451;  // Gauss abscissa 1/sqrt(3)

// Gauss loop rolled (run-time signs) by default: the unrolled form (compile-time
// signs, fewer instructions) needs more registers than a wave64 can hold
// without spilling in FP64, and runs at lower occupancy in FP32.
#ifndef FE_UNROLL64
#define FE_UNROLL64 0
#endif
#ifndef FE_UNROLL32
#define FE_UNROLL32 0
#endif
template <typename T>
struct Unroll { static constexpr bool value = FE_UNROLL32 != 0; };
template <>
struct Unroll<double> { static constexpr bool value = FE_UNROLL64 != 0; };

template <typename T>
struct EC {
    T W;        // (h/2)^3, Gauss weight times Jacobian determinant
    T gs;       // 2/(h*q): physical derivative of a modal sum at a Gauss point
    T Pr, B, eg0, eg1, eg2;
    T inv16h2;  // 1/(16 h^2): |u_e|^2/(16 h^2) is 1/tau_1^2
    T cvisc;    // 16 Pr^2 / h^4 = 1/tau_2^2
    T c16h4;    // 16 / h^4: K^2 * c16h4 = 1/tau_2T^2
    T q0, q1, q2, q3;  // q^|m| / 8 for the modal scaling
    T g1, g2, g3;      // gs q^|m| / 8: modes with |m| >= 1 held premultiplied by gs
    T igs;             // 1 / gs
};

template <typename T>
__device__ __forceinline__ EC<T> make_ec(const Geo &g)
{
    EC<T> c;
    c.W = (T)g.W;
    c.gs = (T)g.gs;
    c.Pr = (T)g.Pr;
    c.B = (T)g.B;
    c.eg0 = (T)g.eg[0];
    c.eg1 = (T)g.eg[1];
    c.eg2 = (T)g.eg[2];
    c.inv16h2 = (T)g.inv16h2;
    c.cvisc = (T)g.cvisc;
    c.c16h4 = (T)g.c16h4;
    c.q0 = (T)0.125;
    c.q1 = (T)(0.125 * QG);
    c.q2 = (T)(0.125 / 3.0);
    c.q3 = (T)(0.125 * QG / 3.0);
    c.g1 = (T)(g.gs * 0.125 * QG);
    c.g2 = (T)(g.gs * 0.125 / 3.0);
    c.g3 = (T)(g.gs * 0.125 * QG / 3.0);
    c.igs = (T)g.igs;
    return c;
}

// Material interpolation (Eqs. conducint, alphaint) and derivatives.
__device__ __forceinline__ double alpha_of(const Geo &g, double y) { return g.amax * (1.0 - y) / (1.0 + g.qa * y); }
__device__ __forceinline__ double K_of(const Geo &g, double y)
{
    return (y * (g.Ck * (1.0 + g.qf) - 1.0) + 1.0) / (g.Ck * (1.0 + g.qf * y));
}
__device__ __forceinline__ double dalpha_of(const Geo &g, double y)
{
    double d = 1.0 + g.qa * y;
    return -g.amax * (1.0 + g.qa) / (d * d);
}
__device__ __forceinline__ double dK_of(const Geo &g, double y)
{
    double d = 1.0 + g.qf * y;
    return (1.0 + g.qf) * (g.Ck - 1.0) / (g.Ck * d * d);
}

__device__ __forceinline__ float rsqrt_t(float a) { return 1.0f / sqrtf(a); }
__device__ __forceinline__ double rsqrt_t(double a) { return 1.0 / sqrt(a); }

// nodal -> scaled modal coefficients: c[m] = q^|m|/8 * sum_a S[a][m] f[a],
// S[a][m] = prod_d s_{a,d}^{m_d}, s = -1 / +1 at the low / high node.
template <typename T>
__device__ __forceinline__ void to_modal(T f[8], const EC<T> &c)
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int bit = 1 << d;
#pragma unroll
        for (int a = 0; a < 8; ++a)
            if (!(a & bit)) {
                T lo = f[a], hi = f[a | bit];
                f[a] = lo + hi;
                f[a | bit] = hi - lo;
            }
    }
    f[0] *= c.q0;
    f[1] *= c.q1; f[2] *= c.q1; f[4] *= c.q1;
    f[3] *= c.q2; f[5] *= c.q2; f[6] *= c.q2;
    f[7] *= c.q3;
}

// As to_modal, with the modes m >= 1 also multiplied by gs (the form eval_pair
// takes): gradients are then plain signed sums of coefficients.
template <typename T>
__device__ __forceinline__ void to_modal_g(T f[8], const EC<T> &c)
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int bit = 1 << d;
#pragma unroll
        for (int a = 0; a < 8; ++a)
            if (!(a & bit)) {
                T lo = f[a], hi = f[a | bit];
                f[a] = lo + hi;
                f[a | bit] = hi - lo;
            }
    }
    f[0] *= c.q0;
    f[1] *= c.g1; f[2] *= c.g1; f[4] *= c.g1;
    f[3] *= c.g2; f[5] *= c.g2; f[6] *= c.g2;
    f[7] *= c.g3;
}

template <bool G, typename T>
__device__ __forceinline__ void to_modal_sel(T f[8], const EC<T> &c)
{
    if (G)
        to_modal_g(f, c);
    else
        to_modal(f, c);
}

// Signs of the Gauss point coordinates (+1 / -1 per direction) and their
// products, either as compile-time constants (fully unrolled Gauss loop) or as
// run-time values (rolled loop, lower register pressure).
template <int G>
struct SgCT {
    static constexpr double sx = (G & 1) ? 1.0 : -1.0;
    static constexpr double sy = (G & 2) ? 1.0 : -1.0;
    static constexpr double sz = (G & 4) ? 1.0 : -1.0;
    static constexpr double sxy = sx * sy, sxz = sx * sz, syz = sy * sz, sxyz = sx * sy * sz;
};

template <typename T>
struct SgRT {
    T sx, sy, sz, sxy, sxz, syz, sxyz;
    __device__ __forceinline__ explicit SgRT(int g)
    {
        sx = (g & 1) ? T(1) : T(-1);
        sy = (g & 2) ? T(1) : T(-1);
        sz = (g & 4) ? T(1) : T(-1);
        sxy = sx * sy;
        sxz = sx * sz;
        syz = sy * sz;
        sxyz = sxy * sz;
    }
};

// Value and physical gradient at the Gauss point with signs SG.
template <typename T, typename SGT>
__device__ __forceinline__ void eval_vg(const SGT &SG, const T m[8], T gs, T &val, T &dx, T &dy,
                                        T &dz)
{
    T t1 = T(SG.sx) * m[1], t2 = T(SG.sy) * m[2], t3 = T(SG.sxy) * m[3], t4 = T(SG.sz) * m[4];
    T t5 = T(SG.sxz) * m[5], t6 = T(SG.syz) * m[6], t7 = T(SG.sxyz) * m[7];
    T ax = (t1 + t3) + (t5 + t7);
    T ay = (t2 + t3) + (t6 + t7);
    T az = (t4 + t5) + (t6 + t7);
    val = ((m[0] + t2) + (t4 + t6)) + ax;
    dx = (T(SG.sx) * gs) * ax;
    dy = (T(SG.sy) * gs) * ay;
    dz = (T(SG.sz) * gs) * az;
}

template <typename T, typename SGT>
__device__ __forceinline__ void eval_g(const SGT &SG, const T m[8], T gs, T &dx, T &dy, T &dz)
{
    T v;
    eval_vg(SG, m, gs, v, dx, dy, dz);
}

// Y[m] += S[g][m] * (c + gs * sum_{d in m} s_d C_d): the modal test-side sum.
template <typename T, typename SGT>
__device__ __forceinline__ void accum(const SGT &SG, T Y[8], T c, T Cx, T Cy, T Cz, T gs)
{
    T px = (T(SG.sx) * gs) * Cx, py = (T(SG.sy) * gs) * Cy, pz = (T(SG.sz) * gs) * Cz;
    T e1 = c + px, e2 = c + py, e4 = c + pz;
    T e3 = e1 + py, e5 = e1 + pz, e6 = e2 + pz, e7 = e3 + pz;
    Y[0] += c;
    Y[1] += T(SG.sx) * e1;
    Y[2] += T(SG.sy) * e2;
    Y[3] += T(SG.sxy) * e3;
    Y[4] += T(SG.sz) * e4;
    Y[5] += T(SG.sxz) * e5;
    Y[6] += T(SG.syz) * e6;
    Y[7] += T(SG.sxyz) * e7;
}

// Run BODY(sg) over the eight Gauss points: unrolled with compile-time signs
// when UNR, else as a rolled loop with run-time signs.
#define FE_GAUSS_LOOP(UNR, T, BODY)                                              \
    if (UNR) {                                                                   \
        { SgCT<0> sg; BODY(sg) } { SgCT<1> sg; BODY(sg) }                        \
        { SgCT<2> sg; BODY(sg) } { SgCT<3> sg; BODY(sg) }                        \
        { SgCT<4> sg; BODY(sg) } { SgCT<5> sg; BODY(sg) }                        \
        { SgCT<6> sg; BODY(sg) } { SgCT<7> sg; BODY(sg) }                        \
    } else {                                                                     \
        _Pragma("unroll 1") for (int g_ = 0; g_ < 8; ++g_) {                     \
            SgRT<T> sg(g_);                                                      \
            BODY(sg)                                                             \
        }                                                                        \
    }

// Gauss points in pairs that differ only in the x sign: the sums over the
// y/z modes are shared by both points.  With the coefficients m[k >= 1] held
// premultiplied by gs (to_modal_g) and (sy, sz) fixed:
//   B0 = m2 + sz m6,  B1 = m3 + sz m7,  C0 = m4 + sy m6,  C1 = m5 + sy m7,
//   A0 = sy B0 + sz m4,  A1 = m1 + sz m5 + sy B1,
//   value = m0 + (A0 + sx A1) / gs,  d/dx = A1,  d/dy = B0 + sx B1,  d/dz = C0 + sx C1,
// 15 operations per field for the two points instead of 2 x 23.
// vm / vp receive {value, d/dx, d/dy, d/dz} at sx = -1 / +1.
#ifndef FE_GP_PAIRS
#define FE_GP_PAIRS 1
#endif
template <typename T>
__device__ __forceinline__ void eval_pair(T sy, T sz, T igs, const T m[8], T vm[4], T vp[4])
{
    const T B0 = fma(sz, m[6], m[2]), B1 = fma(sz, m[7], m[3]);
    const T C0 = fma(sy, m[6], m[4]), C1 = fma(sy, m[7], m[5]);
    const T A1 = fma(sy, B1, fma(sz, m[5], m[1]));
    const T A0 = fma(sy, B0, sz * m[4]);
    const T V0 = fma(igs, A0, m[0]);
    vm[0] = fma(-igs, A1, V0);
    vp[0] = fma(igs, A1, V0);
    vm[1] = vp[1] = A1;
    vm[2] = B0 - B1;
    vp[2] = B0 + B1;
    vm[3] = C0 - C1;
    vp[3] = C0 + C1;
}

// Signs of one point of a pair: sx fixed at compile time, sy and sz at run time.
template <typename T, bool PLUS>
struct SgPair {
    static constexpr double sx = PLUS ? 1.0 : -1.0;
    T sy, sz, sxy, sxz, syz, sxyz;
    __device__ __forceinline__ SgPair(T sy_, T sz_, T syz_)
        : sy(sy_), sz(sz_), sxy(PLUS ? sy_ : -sy_), sxz(PLUS ? sz_ : -sz_), syz(syz_),
          sxyz(PLUS ? syz_ : -syz_)
    {
    }
};

// Run EVAL(sy, sz, syz) (which fills Vm_ and Vp_) and then BODY(sg, Vm_) and
// BODY(sg, Vp_) over the four pairs, as a rolled loop; the points are visited
// in the same order as by FE_GAUSS_LOOP.
#ifndef FE_PAIR_UNROLL
#define FE_PAIR_LOOP_PRAGMA _Pragma("unroll 1")
#else  // compile-time signs; used to count the arithmetic of the element body
#define FE_PAIR_LOOP_PRAGMA _Pragma("unroll")
#endif
//
// BODY(sg, V, ACC) hands each test-side term to ACC(sg, f, c, Cx, Cy, Cz).  With
// FE_PAIR_SUM the terms of both points are kept and the pair is added to the
// modal sums at once (accum_pair); otherwise each point is added as it comes.
#ifndef FE_PAIR_SUM
#define FE_PAIR_SUM 1
#endif
#define FE_ACC_NOW(SG, F, C, X, Y, Z) accum(SG, out[F], C, X, Y, Z, gs);
#define FE_ACC_M(SG, F, C, X, Y, Z) { Pm_[F][0] = C; Pm_[F][1] = X; Pm_[F][2] = Y; Pm_[F][3] = Z; }
#define FE_ACC_P(SG, F, C, X, Y, Z) { Pp_[F][0] = C; Pp_[F][1] = X; Pp_[F][2] = Y; Pp_[F][3] = Z; }
#if FE_PAIR_SUM
#define FE_GAUSS_PAIRS(T, EVAL, BODY)                                            \
    FE_PAIR_LOOP_PRAGMA for (int q_ = 0; q_ < 4; ++q_) {                         \
        const T sy_ = (q_ & 1) ? T(1) : T(-1);                                   \
        const T sz_ = (q_ & 2) ? T(1) : T(-1);                                   \
        const T syz_ = sy_ * sz_;                                                \
        EVAL(sy_, sz_, syz_)                                                     \
        T Pm_[NF][4], Pp_[NF][4];                                                \
        { SgPair<T, false> sg(sy_, sz_, syz_); BODY(sg, Vm_, FE_ACC_M) }          \
        { SgPair<T, true> sg(sy_, sz_, syz_); BODY(sg, Vp_, FE_ACC_P) }           \
        _Pragma("unroll") for (int f_ = 0; f_ < NF; ++f_)                        \
            accum_pair(sy_, sz_, syz_, out[f_], Pm_[f_], Pp_[f_], gs);           \
    }
#else
#define FE_GAUSS_PAIRS(T, EVAL, BODY)                                            \
    FE_PAIR_LOOP_PRAGMA for (int q_ = 0; q_ < 4; ++q_) {                         \
        const T sy_ = (q_ & 1) ? T(1) : T(-1);                                   \
        const T sz_ = (q_ & 2) ? T(1) : T(-1);                                   \
        const T syz_ = sy_ * sz_;                                                \
        EVAL(sy_, sz_, syz_)                                                     \
        { SgPair<T, false> sg(sy_, sz_, syz_); BODY(sg, Vm_, FE_ACC_NOW) }        \
        { SgPair<T, true> sg(sy_, sz_, syz_); BODY(sg, Vp_, FE_ACC_NOW) }         \
    }
#endif

// Test-side sums of a pair of Gauss points that differ only in the x sign (the
// transpose of eval_pair).  pm / pp hold {c, Cx, Cy, Cz} of the points at
// sx = -1 / +1; with _s / _d their sum / difference (p - m) and e = c_d + gs Cx_s:
//   Y0 += c_s             Y1 += e
//   Y2 += sy c_s + gs Cy_s                Y3 += sy e + gs Cy_d
//   Y4 += sz c_s + gs Cz_s                Y5 += sz e + gs Cz_d
//   Y6 += syz c_s + gs (sz Cy_s + sy Cz_s)  Y7 += syz e + gs (sz Cy_d + sy Cz_d)
// which is accum applied to both points (Cx_d drops out).
template <typename T>
__device__ __forceinline__ void accum_pair(T sy, T sz, T syz, T Y[8], const T pm[4],
                                           const T pp[4], T gs)
{
    const T cs = pp[0] + pm[0], cd = pp[0] - pm[0];
    const T xs = pp[1] + pm[1];
    const T ys = pp[2] + pm[2], yd = pp[2] - pm[2];
    const T zs = pp[3] + pm[3], zd = pp[3] - pm[3];
    const T e = fma(gs, xs, cd);
    Y[0] += cs;
    Y[1] += e;
    Y[2] = fma(sy, cs, fma(gs, ys, Y[2]));
    Y[3] = fma(sy, e, fma(gs, yd, Y[3]));
    Y[4] = fma(sz, cs, fma(gs, zs, Y[4]));
    Y[5] = fma(sz, e, fma(gs, zd, Y[5]));
    const T gsy = gs * sy, gsz = gs * sz;  // shared by the five fields of a pair
    Y[6] = fma(gsy, zs, fma(gsz, ys, fma(syz, cs, Y[6])));
    Y[7] = fma(gsy, zd, fma(gsz, yd, fma(syz, e, Y[7])));
}

// Modal test-side sums -> nodal rows: out_a = W sum_m S[a][m] q^|m|/8 Y[m].
template <typename T>
__device__ __forceinline__ void from_modal(T Y[8], const EC<T> &c)
{
    T w0 = c.W * c.q0, w1 = c.W * c.q1, w2 = c.W * c.q2, w3 = c.W * c.q3;
    Y[0] *= w0;
    Y[1] *= w1; Y[2] *= w1; Y[4] *= w1;
    Y[3] *= w2; Y[5] *= w2; Y[6] *= w2;
    Y[7] *= w3;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int bit = 1 << d;
#pragma unroll
        for (int a = 0; a < 8; ++a)
            if (!(a & bit)) {
                T lo = Y[a], hi = Y[a | bit];
                Y[a] = lo - hi;
                Y[a | bit] = lo + hi;
            }
    }
}

// ---- tile staging -------------------------------------------------------------

template <typename T>
struct TileSmem {
    T x[NF][BOXN];
    T v[NF][BOXN];
    T o[NF][BOXN];
};

struct TileIdx {
    int btx, bty, btz, tile;
    int li, lj, lk;      // this thread's element in the tile
    int i, j, k;         // global element
    bool valid;
    int nb[8];           // node-box index of the element's corners
};

#ifndef FE_XCD_REMAP
#define FE_XCD_REMAP 1
#endif
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Map workgroup b to a tile so that every XCD works through a contiguous range
// of tiles: neighbouring tiles, which re-read each other's face nodes, then
// share an L2.  A bijection on [0, n): the last n mod 8 tiles map to themselves.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n >> 3;
    if (b >= (q << 3)) return b;
    return (b & 7) * q + (b >> 3);
}

// blk / nblk: this workgroup's index among the nblk workgroups that cover the
// grid's tiles (blockIdx.x / gridDim.x, or the local index within one problem
// of a batched launch)
__device__ __forceinline__ TileIdx tile_index(const Geo &g, int blk, int nblk)
{
    TileIdx t;
#if FE_XCD_REMAP
    t.tile = xcd_tile(blk, nblk);
#else
    (void)nblk;
    t.tile = blk;
#endif
    t.btx = t.tile % g.ntx;
    int r = t.tile / g.ntx;
    t.bty = r % g.nty;
    t.btz = r / g.nty;
    int th = threadIdx.x;
    t.li = th % TX;
    t.lj = (th / TX) % TY;
    t.lk = th / (TX * TY);
    t.i = t.btx * TX + t.li;
    t.j = t.bty * TY + t.lj;
    t.k = t.btz * TZ + t.lk;
    t.valid = (t.i < g.nx) && (t.j < g.ny) && (t.k < g.nz);
#pragma unroll
    for (int a = 0; a < 8; ++a)
        t.nb[a] = (t.li + (a & 1)) + BX * ((t.lj + ((a >> 1) & 1)) + BY * (t.lk + ((a >> 2) & 1)));
    return t;
}

__device__ __forceinline__ TileIdx tile_index(const Geo &g)
{
    return tile_index(g, (int)blockIdx.x, (int)gridDim.x);
}

__device__ __forceinline__ int64_t gnode(const Geo &g, int I, int J, int K)
{
    return (int64_t)I + (int64_t)(g.nx + 1) * ((int64_t)J + (int64_t)(g.ny + 1) * K);
}

// threadIdx.x hidden from the optimiser (an empty asm statement that claims to
// change it), so that index arithmetic derived from it is not specialised on
// its range.  Used for the FP32 staging loop, where the code generated this way
// measured 18 % faster on the 160x160x320 grid (12 % at 96^3, 2 % at 64^3); the
// FP64 kernels measured 1-2 % slower with it and keep the plain index.
__device__ __forceinline__ int opaque_tid()
{
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Stage one node per thread and iteration (its five values of x and of v,
// and its mask byte): the box position and the global node index are worked
// out once for five values.  Fixed trip count, branch-free loads (nodes
// outside the box or the grid load node 0 and are replaced by 0), all issued
// before the first wait.  The direction may be stored in another type (Tv)
// than the state; it is converted to T as it is staged.
template <typename T, bool HASV, typename Tv = T>
__device__ __forceinline__ void stage_by_node(const Geo &g, const TileIdx &t,
                                              const T *__restrict__ x, const Tv *__restrict__ v,
                                              const uint8_t *__restrict__ nmask, T (*sx)[BOXN],
                                              T (*sv)[BOXN], int tid)
{
    const int tx0 = t.btx * TX, ty0 = t.bty * TY, tz0 = t.btz * TZ;
    constexpr int NIT = (BOXN + NTHR - 1) / NTHR;
    T xv[NIT][NF], vv[NIT][NF];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int nb = tid + it * NTHR;
        const int lx = nb % BX, r = nb / BX, ly = r % BY, lz = r / BY;
        const int I = tx0 + lx, J = ty0 + ly, K = tz0 + lz;
        const bool in = nb < BOXN && I <= g.nx && J <= g.ny && K <= g.nz;
        const int64_t gn = in ? gnode(g, I, J, K) : 0;
        const T *xp = x + NF * gn;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const T xl = xp[f];
            xv[it][f] = in ? xl : T(0);
        }
        if (HASV) {
            const Tv *vp = v + NF * gn;
            const int m = in ? (int)nmask[gn] : 0x1f;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const T vl = (T)vp[f];
                vv[it][f] = ((m >> f) & 1) ? T(0) : vl;
            }
        }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int nb = tid + it * NTHR;
        if (nb < BOXN) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                sx[f][nb] = xv[it][f];
                if (HASV) sv[f][nb] = vv[it][f];
            }
        }
    }
}

// Stage one value (node and field) per thread and iteration, fixed trip count,
// branch-free as above.
template <typename T, bool HASV, typename Tv = T>
__device__ __forceinline__ void stage_by_value(const Geo &g, const TileIdx &t,
                                               const T *__restrict__ x, const Tv *__restrict__ v,
                                               const uint8_t *__restrict__ nmask, T (*sx)[BOXN],
                                               T (*sv)[BOXN], int tid)
{
    const int tx0 = t.btx * TX, ty0 = t.bty * TY, tz0 = t.btz * TZ;
    constexpr int NIT = (BOXN * NF + NTHR - 1) / NTHR;
    T xv[NIT], vv[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = tid + it * NTHR;
        const int nb = idx / NF, f = idx - nb * NF;
        const int lx = nb % BX, r = nb / BX, ly = r % BY, lz = r / BY;
        const int I = tx0 + lx, J = ty0 + ly, K = tz0 + lz;
        const bool in = idx < BOXN * NF && I <= g.nx && J <= g.ny && K <= g.nz;
        const int64_t gn = in ? gnode(g, I, J, K) : 0;
        const T xl = x[NF * gn + f];
        xv[it] = in ? xl : T(0);
        vv[it] = T(0);
        if (HASV) {
            const T vl = (T)v[NF * gn + f];
            const int m = nmask[gn];
            const bool keep = in & (((m >> f) & 1) == 0);
            vv[it] = keep ? vl : T(0);
        }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int idx = tid + it * NTHR;
        if (idx < BOXN * NF) {
            int nb = idx / NF, f = idx - nb * NF;
            sx[f][nb] = xv[it];
            if (HASV) sv[f][nb] = vv[it];
        }
    }
}

// Stage the node box of x (and of the masked direction v) in LDS; zero the
// output accumulator.  The FP32 kernels stage by node: that measured 4-5 %
// faster for the FP32 J v element pass (64^3: 31.2 -> 29.9 us, 160x160x320:
// 709 -> 675 us).  The FP64 kernels stage by value: by node, J v and J^T w did
// not change and the residual, whose body then no longer fits two waves per
// SIMD, ran 18-23 % slower.
template <typename T, int NVO, bool HASV, typename Tv = T>
__device__ __forceinline__ void stage(const Geo &g, const TileIdx &t, const T *__restrict__ x,
                                      const Tv *__restrict__ v, const uint8_t *__restrict__ nmask,
                                      T (*sx)[BOXN], T (*sv)[BOXN], T *so)
{
    if constexpr (sizeof(T) == 4)
        stage_by_node<T, HASV, Tv>(g, t, x, v, nmask, sx, sv, opaque_tid());
    else
        stage_by_value<T, HASV, Tv>(g, t, x, v, nmask, sx, sv, (int)threadIdx.x);
    if (NVO > 0)
        for (int idx = threadIdx.x; idx < BOXN * NVO; idx += NTHR) so[idx] = T(0);
}

// Is node coordinate I (local lx) shared with the neighbouring tile in that direction?
__device__ __forceinline__ bool shared_dir(int l, int I, int n, int T_)
{
    return (l == 0 && I > 0) || (l == T_ && I < n);
}

// ---- element bodies -------------------------------------------------------------

// Residual rows of one element (Galerkin + SUPG + PSPG, see header comment).
template <typename T, bool UNR>
__device__ __forceinline__ void elem_residual(const EC<T> &c, const T (*sx)[BOXN], const int nb[8],
                                              T alpha, T Kc, T s, T out[NF][8])
{
    T mu[3][8], mp[8], mT[8];
    T U2 = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            T xa = sx[i][nb[a]];
            U2 += xa * xa;
            mu[i][a] = xa;
        }
        to_modal(mu[i], c);
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        mp[a] = sx[3][nb[a]];
        mT[a] = sx[4][nb[a]];
    }
    to_modal(mp, c);
    to_modal(mT, c);
    const T tau = rsqrt_t(U2 * c.inv16h2 + c.cvisc + alpha * alpha);
    const T tauT = rsqrt_t(U2 * c.inv16h2 + Kc * Kc * c.c16h4);
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int m = 0; m < 8; ++m) out[f][m] = T(0);
    const T gs = c.gs;
// V[f] = {value, d/dx, d/dy, d/dz} for f = u, v, w, p, T.
#define FE_RES_EVAL1(SG)                                                                      \
    T V1_[5][4];                                                                             \
    _Pragma("unroll") for (int i = 0; i < 3; ++i)                                            \
        eval_vg(SG, mu[i], gs, V1_[i][0], V1_[i][1], V1_[i][2], V1_[i][3]);                   \
    eval_vg(SG, mp, gs, V1_[3][0], V1_[3][1], V1_[3][2], V1_[3][3]);                          \
    eval_vg(SG, mT, gs, V1_[4][0], V1_[4][1], V1_[4][2], V1_[4][3]);
#define FE_RES_POINT(SG, V)                                                                   \
    {                                                                                        \
        T u[3], Gd[3][3];                                                                    \
        _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                      \
            u[i] = V[i][0];                                                                  \
            _Pragma("unroll") for (int d = 0; d < 3; ++d) Gd[i][d] = V[i][1 + d];            \
        }                                                                                    \
        const T pv = V[3][0], gp0 = V[3][1], gp1 = V[3][2], gp2 = V[3][3];                   \
        const T Tv = V[4][0], gT0 = V[4][1], gT1 = V[4][2], gT2 = V[4][3];                   \
        T conv[3], rM[3];                                                                    \
        const T egv[3] = {c.eg0, c.eg1, c.eg2};                                              \
        const T gpv[3] = {gp0, gp1, gp2};                                                    \
        _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                      \
            conv[i] = u[0] * Gd[i][0] + u[1] * Gd[i][1] + u[2] * Gd[i][2];                   \
            T gal = conv[i] + alpha * u[i] + c.B * egv[i] * Tv;                              \
            rM[i] = gal + gpv[i];                                                            \
            conv[i] = gal;                                                                   \
        }                                                                                    \
        T rT = u[0] * gT0 + u[1] * gT1 + u[2] * gT2 - s;                                     \
        _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                      \
            T tr = tau * rM[i];                                                              \
            T C0 = c.Pr * (Gd[i][0] + Gd[0][i]) + u[0] * tr;                                 \
            T C1 = c.Pr * (Gd[i][1] + Gd[1][i]) + u[1] * tr;                                 \
            T C2 = c.Pr * (Gd[i][2] + Gd[2][i]) + u[2] * tr;                                 \
            if (i == 0) C0 -= pv;                                                            \
            if (i == 1) C1 -= pv;                                                            \
            if (i == 2) C2 -= pv;                                                            \
            accum(SG, out[i], conv[i], C0, C1, C2, gs);                                       \
        }                                                                                    \
        accum(SG, out[3], Gd[0][0] + Gd[1][1] + Gd[2][2], tau * rM[0], tau * rM[1],           \
                 tau * rM[2], gs);                                                           \
        T trT = tauT * rT;                                                                   \
        accum(SG, out[4], rT, Kc * gT0 + u[0] * trT, Kc * gT1 + u[1] * trT,                   \
                 Kc * gT2 + u[2] * trT, gs);                                                 \
    }
// One point at a time: the paired form needs more than 256 registers here,
// which halves the residual's occupancy (2 -> 1 workgroup per CU); it ran 24 %
// slower.
#define FE_RES_GP(SG) { FE_RES_EVAL1(SG) FE_RES_POINT(SG, V1_) }
    FE_GAUSS_LOOP(UNR, T, FE_RES_GP)
#undef FE_RES_EVAL1
#undef FE_RES_POINT
#undef FE_RES_GP
#pragma unroll
    for (int f = 0; f < NF; ++f) from_modal(out[f], c);
}

// Directional derivative J_e v_e (exact linearisation, including d tau).
// xs(f, a), vs(f, a): the state and the direction at corner a, field f.
template <typename T, bool UNR, typename XS, typename VS>
__device__ __forceinline__ void elem_jv(const EC<T> &c, XS xs, VS vs, T alpha, T Kc, T s,
                                        T out[NF][8])
{
    constexpr bool PG = !UNR && FE_GP_PAIRS;  // paired Gauss points: gs-scaled modes
    T mu[3][8], md[3][8], mp[8], mT[8], mdp[8], mdT[8];
    T U2 = T(0), udu = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            T xa = xs(i, a), va = vs(i, a);
            U2 += xa * xa;
            udu += xa * va;
            mu[i][a] = xa;
            md[i][a] = va;
        }
        to_modal_sel<PG>(mu[i], c);
        to_modal_sel<PG>(md[i], c);
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        mp[a] = xs(3, a);
        mT[a] = xs(4, a);
        mdp[a] = vs(3, a);
        mdT[a] = vs(4, a);
    }
    to_modal_sel<PG>(mp, c);
    to_modal_sel<PG>(mT, c);
    to_modal_sel<PG>(mdp, c);
    to_modal_sel<PG>(mdT, c);
    const T tau = rsqrt_t(U2 * c.inv16h2 + c.cvisc + alpha * alpha);
    const T tauT = rsqrt_t(U2 * c.inv16h2 + Kc * Kc * c.c16h4);
    const T dtau = -(tau * tau * tau) * udu * c.inv16h2;
    const T dtauT = -(tauT * tauT * tauT) * udu * c.inv16h2;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int m = 0; m < 8; ++m) out[f][m] = T(0);
    const T gs = c.gs;
// Field values at one Gauss point, V[f] = {value, d/dx, d/dy, d/dz} for
// f = u, v, w, du, dv, dw, p, T, dp, dT.
#define FE_JV_EVAL1(SG)                                                                       \
    T V1_[10][4];                                                                            \
    _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                          \
        eval_vg(SG, mu[i], gs, V1_[i][0], V1_[i][1], V1_[i][2], V1_[i][3]);                   \
        eval_vg(SG, md[i], gs, V1_[3 + i][0], V1_[3 + i][1], V1_[3 + i][2], V1_[3 + i][3]);   \
    }                                                                                        \
    eval_vg(SG, mp, gs, V1_[6][0], V1_[6][1], V1_[6][2], V1_[6][3]);                          \
    eval_vg(SG, mT, gs, V1_[7][0], V1_[7][1], V1_[7][2], V1_[7][3]);                          \
    eval_vg(SG, mdp, gs, V1_[8][0], V1_[8][1], V1_[8][2], V1_[8][3]);                         \
    eval_vg(SG, mdT, gs, V1_[9][0], V1_[9][1], V1_[9][2], V1_[9][3]);
#define FE_JV_EVAL2(SY, SZ, SYZ)                                                              \
    T Vm_[10][4], Vp_[10][4];                                                                \
    _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                          \
        eval_pair(SY, SZ, c.igs, mu[i], Vm_[i], Vp_[i]);                                    \
        eval_pair(SY, SZ, c.igs, md[i], Vm_[3 + i], Vp_[3 + i]);                            \
    }                                                                                        \
    eval_pair(SY, SZ, c.igs, mp, Vm_[6], Vp_[6]);                                           \
    eval_pair(SY, SZ, c.igs, mT, Vm_[7], Vp_[7]);                                           \
    eval_pair(SY, SZ, c.igs, mdp, Vm_[8], Vp_[8]);                                          \
    eval_pair(SY, SZ, c.igs, mdT, Vm_[9], Vp_[9]);
#define FE_JV_POINT(SG, V, ACC)                                                                  \
    {                                                                                        \
        T u[3], Gd[3][3], du[3], dG[3][3];                                                   \
        _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                      \
            u[i] = V[i][0];                                                                  \
            du[i] = V[3 + i][0];                                                             \
            _Pragma("unroll") for (int d = 0; d < 3; ++d) {                                  \
                Gd[i][d] = V[i][1 + d];                                                      \
                dG[i][d] = V[3 + i][1 + d];                                                  \
            }                                                                                \
        }                                                                                    \
        const T gp[3] = {V[6][1], V[6][2], V[6][3]};                                         \
        const T Tv = V[7][0], gT[3] = {V[7][1], V[7][2], V[7][3]};                           \
        const T dpv = V[8][0], gdp[3] = {V[8][1], V[8][2], V[8][3]};                         \
        const T dTv = V[9][0], gdT[3] = {V[9][1], V[9][2], V[9][3]};                         \
        const T egv[3] = {c.eg0, c.eg1, c.eg2};                                              \
        T rM[3], dgal[3], A[3], Bm[3];                                                       \
        _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                      \
            T conv = u[0] * Gd[i][0] + u[1] * Gd[i][1] + u[2] * Gd[i][2];                    \
            T dconv = du[0] * Gd[i][0] + du[1] * Gd[i][1] + du[2] * Gd[i][2]                 \
                    + u[0] * dG[i][0] + u[1] * dG[i][1] + u[2] * dG[i][2];                   \
            rM[i] = conv + gp[i] + alpha * u[i] + c.B * egv[i] * Tv;                         \
            dgal[i] = dconv + alpha * du[i] + c.B * egv[i] * dTv;                            \
            T drM = dgal[i] + gdp[i];                                                        \
            A[i] = dtau * rM[i] + tau * drM;                                                 \
            Bm[i] = tau * rM[i];                                                             \
        }                                                                                    \
        T rT = u[0] * gT[0] + u[1] * gT[1] + u[2] * gT[2] - s;                               \
        T drT = du[0] * gT[0] + du[1] * gT[1] + du[2] * gT[2]                                \
              + u[0] * gdT[0] + u[1] * gdT[1] + u[2] * gdT[2];                               \
        _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                      \
            T C0 = c.Pr * (dG[i][0] + dG[0][i]) + u[0] * A[i] + du[0] * Bm[i];               \
            T C1 = c.Pr * (dG[i][1] + dG[1][i]) + u[1] * A[i] + du[1] * Bm[i];               \
            T C2 = c.Pr * (dG[i][2] + dG[2][i]) + u[2] * A[i] + du[2] * Bm[i];               \
            if (i == 0) C0 -= dpv;                                                           \
            if (i == 1) C1 -= dpv;                                                           \
            if (i == 2) C2 -= dpv;                                                           \
            ACC(SG, i, dgal[i], C0, C1, C2)                                                  \
        }                                                                                    \
        ACC(SG, 3, dG[0][0] + dG[1][1] + dG[2][2], A[0], A[1], A[2])                         \
        T AT = dtauT * rT + tauT * drT, BT = tauT * rT;                                      \
        ACC(SG, 4, drT, Kc * gdT[0] + u[0] * AT + du[0] * BT,                                 \
            Kc * gdT[1] + u[1] * AT + du[1] * BT, Kc * gdT[2] + u[2] * AT + du[2] * BT)      \
    }
#define FE_JV_GP(SG) { FE_JV_EVAL1(SG) FE_JV_POINT(SG, V1_, FE_ACC_NOW) }
    if (UNR || !FE_GP_PAIRS) {
        FE_GAUSS_LOOP(UNR, T, FE_JV_GP)
    } else {
        FE_GAUSS_PAIRS(T, FE_JV_EVAL2, FE_JV_POINT)
    }
#undef FE_JV_EVAL1
#undef FE_JV_EVAL2
#undef FE_JV_POINT
#undef FE_JV_GP
#pragma unroll
    for (int f = 0; f < NF; ++f) from_modal(out[f], c);
}

// Transposed product J_e^T w_e in one reverse pass with recomputed state:
// adjoint test fields Lambda (velocity rows), Pi (pressure rows), Theta
// (temperature rows) are interpolated from w_e; the multipliers of the varied
// strong residuals are mu = tau (u.grad Lambda + grad Pi) and muT = tauT u.grad Theta;
// the element-level tau variation is applied after the Gauss loop.
template <typename T, bool UNR>
__device__ __forceinline__ void elem_jtv(const EC<T> &c, const T (*sx)[BOXN], const T (*sv)[BOXN],
                                         const int nb[8], T alpha, T Kc, T s, T out[NF][8])
{
    constexpr bool PG = !UNR && FE_GP_PAIRS;  // paired Gauss points: gs-scaled modes
    T mu[3][8], mL[3][8], mp[8], mT[8], mP[8], mTh[8];
    T U2 = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            T xa = sx[i][nb[a]];
            U2 += xa * xa;
            mu[i][a] = xa;
            mL[i][a] = sv[i][nb[a]];
        }
        to_modal_sel<PG>(mu[i], c);
        to_modal_sel<PG>(mL[i], c);
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        mp[a] = sx[3][nb[a]];
        mT[a] = sx[4][nb[a]];
        mP[a] = sv[3][nb[a]];
        mTh[a] = sv[4][nb[a]];
    }
    to_modal_sel<PG>(mp, c);
    to_modal_sel<PG>(mT, c);
    to_modal_sel<PG>(mP, c);
    to_modal_sel<PG>(mTh, c);
    const T tau = rsqrt_t(U2 * c.inv16h2 + c.cvisc + alpha * alpha);
    const T tauT = rsqrt_t(U2 * c.inv16h2 + Kc * Kc * c.c16h4);
    T Aacc = T(0), ATacc = T(0);
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int m = 0; m < 8; ++m) out[f][m] = T(0);
    const T gs = c.gs;
// V[f] = {value, d/dx, d/dy, d/dz} for f = u, v, w, Lambda (3), p, T, Pi, Theta.
#define FE_JTV_EVAL1(SG)                                                                      \
    T V1_[10][4];                                                                            \
    _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                          \
        eval_vg(SG, mu[i], gs, V1_[i][0], V1_[i][1], V1_[i][2], V1_[i][3]);                   \
        eval_vg(SG, mL[i], gs, V1_[3 + i][0], V1_[3 + i][1], V1_[3 + i][2], V1_[3 + i][3]);   \
    }                                                                                        \
    eval_vg(SG, mp, gs, V1_[6][0], V1_[6][1], V1_[6][2], V1_[6][3]);                          \
    eval_vg(SG, mT, gs, V1_[7][0], V1_[7][1], V1_[7][2], V1_[7][3]);                          \
    eval_vg(SG, mP, gs, V1_[8][0], V1_[8][1], V1_[8][2], V1_[8][3]);                          \
    eval_vg(SG, mTh, gs, V1_[9][0], V1_[9][1], V1_[9][2], V1_[9][3]);
#define FE_JTV_EVAL2(SY, SZ, SYZ)                                                             \
    T Vm_[10][4], Vp_[10][4];                                                                \
    _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                          \
        eval_pair(SY, SZ, c.igs, mu[i], Vm_[i], Vp_[i]);                                    \
        eval_pair(SY, SZ, c.igs, mL[i], Vm_[3 + i], Vp_[3 + i]);                            \
    }                                                                                        \
    eval_pair(SY, SZ, c.igs, mp, Vm_[6], Vp_[6]);                                           \
    eval_pair(SY, SZ, c.igs, mT, Vm_[7], Vp_[7]);                                           \
    eval_pair(SY, SZ, c.igs, mP, Vm_[8], Vp_[8]);                                           \
    eval_pair(SY, SZ, c.igs, mTh, Vm_[9], Vp_[9]);
#define FE_JTV_POINT(SG, V, ACC)                                                                 \
    {                                                                                        \
        T u[3], Gd[3][3], L[3], LG[3][3];                                                    \
        _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                      \
            u[i] = V[i][0];                                                                  \
            L[i] = V[3 + i][0];                                                              \
            _Pragma("unroll") for (int d = 0; d < 3; ++d) {                                  \
                Gd[i][d] = V[i][1 + d];                                                      \
                LG[i][d] = V[3 + i][1 + d];                                                  \
            }                                                                                \
        }                                                                                    \
        const T gp[3] = {V[6][1], V[6][2], V[6][3]};                                         \
        const T Tv = V[7][0], gT[3] = {V[7][1], V[7][2], V[7][3]};                           \
        const T Pv = V[8][0], gP[3] = {V[8][1], V[8][2], V[8][3]};                           \
        const T Th = V[9][0], gTh[3] = {V[9][1], V[9][2], V[9][3]};                          \
        const T egv[3] = {c.eg0, c.eg1, c.eg2};                                              \
        T rM[3], uL[3], mI[3], LM[3];                                                        \
        _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                      \
            rM[i] = u[0] * Gd[i][0] + u[1] * Gd[i][1] + u[2] * Gd[i][2] + gp[i]             \
                  + alpha * u[i] + c.B * egv[i] * Tv;                                        \
            uL[i] = u[0] * LG[i][0] + u[1] * LG[i][1] + u[2] * LG[i][2];                     \
            T q = uL[i] + gP[i];                                                             \
            mI[i] = tau * q;                                                                 \
            Aacc += q * rM[i];                                                               \
            LM[i] = L[i] + mI[i];                                                            \
        }                                                                                    \
        T rT = u[0] * gT[0] + u[1] * gT[1] + u[2] * gT[2] - s;                               \
        T uTh = u[0] * gTh[0] + u[1] * gTh[1] + u[2] * gTh[2];                               \
        ATacc += uTh * rT;                                                                   \
        T ThM = Th + tauT * uTh;                                                             \
        T trT = tauT * rT;                                                                   \
        _Pragma("unroll") for (int j = 0; j < 3; ++j) {                                      \
            T cj = LM[0] * Gd[0][j] + LM[1] * Gd[1][j] + LM[2] * Gd[2][j] + alpha * LM[j]    \
                 + tau * (LG[0][j] * rM[0] + LG[1][j] * rM[1] + LG[2][j] * rM[2])            \
                 + trT * gTh[j] + ThM * gT[j];                                               \
            T C0 = LM[j] * u[0] + c.Pr * (LG[j][0] + LG[0][j]);                              \
            T C1 = LM[j] * u[1] + c.Pr * (LG[j][1] + LG[1][j]);                              \
            T C2 = LM[j] * u[2] + c.Pr * (LG[j][2] + LG[2][j]);                              \
            if (j == 0) C0 += Pv;                                                            \
            if (j == 1) C1 += Pv;                                                            \
            if (j == 2) C2 += Pv;                                                            \
            ACC(SG, j, cj, C0, C1, C2)                                                       \
        }                                                                                    \
        ACC(SG, 3, -(LG[0][0] + LG[1][1] + LG[2][2]), mI[0], mI[1], mI[2])                   \
        ACC(SG, 4, c.B * (egv[0] * LM[0] + egv[1] * LM[1] + egv[2] * LM[2]),                  \
            Kc * gTh[0] + ThM * u[0], Kc * gTh[1] + ThM * u[1], Kc * gTh[2] + ThM * u[2])    \
    }
#define FE_JTV_GP(SG) { FE_JTV_EVAL1(SG) FE_JTV_POINT(SG, V1_, FE_ACC_NOW) }
    if (UNR || !FE_GP_PAIRS) {
        FE_GAUSS_LOOP(UNR, T, FE_JTV_GP)
    } else {
        FE_GAUSS_PAIRS(T, FE_JTV_EVAL2, FE_JTV_POINT)
    }
#undef FE_JTV_EVAL1
#undef FE_JTV_EVAL2
#undef FE_JTV_POINT
#undef FE_JTV_GP
#pragma unroll
    for (int f = 0; f < NF; ++f) from_modal(out[f], c);
    // d tau / d u_e and d tauT / d u_e contributions: -(tau^3 A + tauT^3 A_T) u_e / (16 h^2)
    const T coef = -(tau * tau * tau * Aacc + tauT * tauT * tauT * ATacc) * c.W * c.inv16h2;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int a = 0; a < 8; ++a) out[i][a] += coef * sx[i][nb[a]];
}

// ---- tile kernel: element loop + ordered LDS accumulation + face slots ---------

// Tv: the direction's storage type (default the state's); it is staged as Tin.
template <typename Tin, typename Tout, int OP, typename Tv = Tin>
__device__ __forceinline__ void elem_tile(const Geo &g, const Tin *__restrict__ x,
                                          const Tv *__restrict__ v,
                                          const double *__restrict__ gamma,
                                          const double *__restrict__ src,
                                          const uint8_t *__restrict__ nmask,
                                          Tout *__restrict__ out, Tout *__restrict__ slots, int blk,
                                          int nblk)
{
    using T = Tin;
    __shared__ TileSmem<T> S;
    const TileIdx t = tile_index(g, blk, nblk);
    stage<T, NF, OP != OP_RES, Tv>(g, t, x, (OP == OP_RES) ? nullptr : v, nmask, S.x,
                 (OP == OP_RES) ? nullptr : S.v, &S.o[0][0]);
    __syncthreads();

    T R[NF][8];
    if (t.valid) {
        const EC<T> c = make_ec<T>(g);
        const int64_t e = (int64_t)t.i + (int64_t)g.nx * ((int64_t)t.j + (int64_t)g.ny * t.k);
        const double y = gamma[e];
        const T alpha = (T)alpha_of(g, y), Kc = (T)K_of(g, y), s = (T)src[e];
        constexpr bool UNR = Unroll<T>::value;
        if (OP == OP_RES)
            elem_residual<T, UNR>(c, S.x, t.nb, alpha, Kc, s, R);
        else if (OP == OP_JV)
            elem_jv<T, UNR>(
                c, [&](int f, int a) { return S.x[f][t.nb[a]]; },
                [&](int f, int a) { return S.v[f][t.nb[a]]; }, alpha, Kc, s, R);
        else
            elem_jtv<T, UNR>(c, S.x, S.v, t.nb, alpha, Kc, s, R);
    }
    // ordered accumulation: in sub-step a every thread adds its corner-a row
    // to a distinct node of the box
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        if (t.valid) {
#pragma unroll
            for (int f = 0; f < NF; ++f) S.o[f][t.nb[a]] += R[f][a];
        }
        __syncthreads();
    }
    // write-out: complete nodes to out, shared ones to the tile's slots
    const int tx0 = t.btx * TX, ty0 = t.bty * TY, tz0 = t.btz * TZ;
    // fixed trip count: the node-mask loads of all of this thread's nodes are
    // issued before the first is waited for
    constexpr int NWO = (BOXN + NTHR - 1) / NTHR;
    int64_t gnw[NWO];
    int mw[NWO];
    bool own[NWO], shw[NWO];
#pragma unroll
    for (int it = 0; it < NWO; ++it) {
        const int nb = threadIdx.x + it * NTHR;
        const int lx = nb % BX, r = nb / BX, ly = r % BY, lz = r / BY;
        const int I = tx0 + lx, J = ty0 + ly, K = tz0 + lz;
        const bool in = nb < BOXN && I <= g.nx && J <= g.ny && K <= g.nz;
        const bool sh = shared_dir(lx, I, g.nx, TX) | shared_dir(ly, J, g.ny, TY) |
                        shared_dir(lz, K, g.nz, TZ);
        shw[it] = in & sh;
        own[it] = in & !sh;
        gnw[it] = own[it] ? gnode(g, I, J, K) : 0;
        mw[it] = nmask[gnw[it]];
    }
#pragma unroll
    for (int it = 0; it < NWO; ++it) {
        const int nb = threadIdx.x + it * NTHR;
        if (shw[it]) {
            Tout *sl = slots + ((int64_t)t.tile * BOXN + nb) * NF;
#pragma unroll
            for (int f = 0; f < NF; ++f) sl[f] = (Tout)S.o[f][nb];
        } else if (own[it]) {
            const int64_t gn = gnw[it];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                Tout val = (Tout)S.o[f][nb];
                if ((mw[it] >> f) & 1) val = (OP == OP_RES) ? Tout(0) : (Tout)v[NF * gn + f];
                out[NF * gn + f] = val;
            }
        }
    }
}

template <typename Tin, typename Tout, int OP>
__global__ __launch_bounds__(NTHR) void k_elem(Geo g, const Tin *__restrict__ x,
                                               const Tin *__restrict__ v,
                                               const double *__restrict__ gamma,
                                               const double *__restrict__ src,
                                               const uint8_t *__restrict__ nmask,
                                               Tout *__restrict__ out, Tout *__restrict__ slots)
{
    elem_tile<Tin, Tout, OP>(g, x, v, gamma, src, nmask, out, slots, (int)blockIdx.x,
                             (int)gridDim.x);
}

// The FP64 operator (J v or J^T w) with the direction stored in FP32.
template <int OP>
__global__ __launch_bounds__(NTHR) void k_elem_dir32(Geo g, const double *__restrict__ x,
                                                     const float *__restrict__ v,
                                                     const double *__restrict__ gamma,
                                                     const double *__restrict__ src,
                                                     const uint8_t *__restrict__ nmask,
                                                     double *__restrict__ out,
                                                     double *__restrict__ slots)
{
    elem_tile<double, double, OP, float>(g, x, v, gamma, src, nmask, out, slots,
                                         (int)blockIdx.x, (int)gridDim.x);
}

// Tiles containing node coordinate I along one direction, in increasing order.
// With one tile, the second entry repeats the first (a valid address for
// unrolled loads whose term is dropped).
__device__ __forceinline__ int tiles_of(int I, int n, int T_, int nt, int tl[2], int ll[2])
{
    if (I % T_ == 0 && I > 0 && I < n) {
        tl[0] = I / T_ - 1; ll[0] = T_;
        tl[1] = I / T_;     ll[1] = 0;
        return 2;
    }
    int t = I / T_;
    if (t >= nt) t = nt - 1;
    tl[0] = t; ll[0] = I - t * T_;
    tl[1] = tl[0]; ll[1] = ll[0];
    return 1;
}

// Sum of the slot partials of node (I, J, K) over its cz x cy x cx tiles in the
// fixed tile order (z, then y, then x).  The 2 x 2 x 2 candidates are unrolled,
// absent ones loading nothing and adding zero, so that the slot loads of all
// present tiles are in flight together.
template <typename T>
__device__ __forceinline__ void sum_slots5(const Geo &g, const T *__restrict__ slots, const int tx[2],
                                           const int lx[2], const int ty[2], const int ly[2],
                                           const int tz[2], const int lz[2], int cx, int cy, int cz,
                                           T acc[NF])
{
#pragma unroll
    for (int q = 0; q < NF; ++q) acc[q] = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                const bool use = (a < cz) && (b < cy) && (cc < cx);
                const int64_t tile = tx[cc] + (int64_t)g.ntx * (ty[b] + (int64_t)g.nty * tz[a]);
                const int nb = lx[cc] + BX * (ly[b] + BY * lz[a]);
                const T *sl = slots + (tile * BOXN + nb) * NF;
                T v[NF];
#pragma unroll
                for (int q = 0; q < NF; ++q) v[q] = T(0);
                if (use) {
#pragma unroll
                    for (int q = 0; q < NF; ++q) v[q] = sl[q];
                }
#pragma unroll
                for (int q = 0; q < NF; ++q) acc[q] += v[q];
            }
}

// Sum the slot partials of nodes shared between tiles, in a fixed tile order.
template <typename Tv, typename Tout, int NV, int OP>
__device__ __forceinline__ void combine_nodes(const Geo &g, const Tout *__restrict__ slots,
                                              const uint8_t *__restrict__ nmask,
                                              const Tv *__restrict__ v, Tout *__restrict__ out,
                                              unsigned blk)
{
    const int64_t nn = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    const int64_t gn = (int64_t)blk * blockDim.x + threadIdx.x;
    if (gn >= nn) return;
    const int I = (int)(gn % (g.nx + 1));
    const int64_t r = gn / (g.nx + 1);
    const int J = (int)(r % (g.ny + 1));
    const int K = (int)(r / (g.ny + 1));
    int tx[2], lx[2], ty[2], ly[2], tz[2], lz[2];
    int cx = tiles_of(I, g.nx, TX, g.ntx, tx, lx);
    int cy = tiles_of(J, g.ny, TY, g.nty, ty, ly);
    int cz = tiles_of(K, g.nz, TZ, g.ntz, tz, lz);
    if (cx == 1 && cy == 1 && cz == 1) return;  // written by its only tile
    Tout acc[NV];
    if (NV == NF) {
        sum_slots5<Tout>(g, slots, tx, lx, ty, ly, tz, lz, cx, cy, cz, acc);
    } else {
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = Tout(0);
        for (int a = 0; a < cz; ++a)
            for (int b = 0; b < cy; ++b)
                for (int cc = 0; cc < cx; ++cc) {
                    int64_t tile = tx[cc] + (int64_t)g.ntx * (ty[b] + (int64_t)g.nty * tz[a]);
                    int nb = lx[cc] + BX * (ly[b] + BY * lz[a]);
                    const Tout *sl = slots + (tile * BOXN + nb) * NV;
#pragma unroll
                    for (int q = 0; q < NV; ++q) acc[q] += sl[q];
                }
    }
    const uint8_t m = nmask[gn];
    if (NV == NF) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            Tout val = acc[f];
            if ((m >> f) & 1) val = (OP == OP_RES) ? Tout(0) : (Tout)v[NF * gn + f];
            out[NF * gn + f] = val;
        }
    } else {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int f2 = 0; f2 < NF; ++f2) {
                Tout val = acc[f * NF + f2];
                if (((m >> f) & 1) || ((m >> f2) & 1)) val = (f == f2) ? Tout(1) : Tout(0);
                out[gn * 25 + f * NF + f2] = val;
            }
    }
}

template <typename Tv, typename Tout, int NV, int OP>
__global__ __launch_bounds__(256) void k_combine(Geo g, const Tout *__restrict__ slots,
                                                 const uint8_t *__restrict__ nmask,
                                                 const Tv *__restrict__ v, Tout *__restrict__ out)
{
    combine_nodes<Tv, Tout, NV, OP>(g, slots, nmask, v, out, blockIdx.x);
}

// The shared-node pass fused with one damped block-Jacobi sweep of the
// multigrid smoother: t = J x is completed per node exactly as k_combine does
// (rows of a node inside one tile were written to t by the element pass), and
// x += omega D^{-1} (b - t) (D^{-T} for the transposed operator) is applied at
// once, so t is never written for shared nodes nor read back.  Each thread
// reads and writes only its own node of x.
template <typename T, int OP>
__device__ __forceinline__ void combine_smooth_nodes(const Geo &g, const T *__restrict__ slots,
                                                     const uint8_t *__restrict__ nmask,
                                                     const T *__restrict__ t,
                                                     const T *__restrict__ D,
                                                     const T *__restrict__ b, T *x, T omega,
                                                     unsigned blk)
{
    const int64_t nn = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    __shared__ T sD[256 * 25];
    const int64_t n0 = (int64_t)blk * 256;
    const T *Dn = stage_blocks256(D, n0, nn, sD);
    const int64_t gn = n0 + threadIdx.x;
    if (gn >= nn) return;
    const int I = (int)(gn % (g.nx + 1));
    const int64_t r = gn / (g.nx + 1);
    const int J = (int)(r % (g.ny + 1));
    const int K = (int)(r / (g.ny + 1));
    int tx[2], lx[2], ty[2], ly[2], tz[2], lz[2];
    const int cx = tiles_of(I, g.nx, TX, g.ntx, tx, lx);
    const int cy = tiles_of(J, g.ny, TY, g.nty, ty, ly);
    const int cz = tiles_of(K, g.nz, TZ, g.ntz, tz, lz);
    T tv[NF];
    if (cx == 1 && cy == 1 && cz == 1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) tv[f] = t[NF * gn + f];
    } else {
        sum_slots5<T>(g, slots, tx, lx, ty, ly, tz, lz, cx, cy, cz, tv);
        const uint8_t m = nmask[gn];
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if ((m >> f) & 1) tv[f] = x[NF * gn + f];
    }
    T rr[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) rr[f] = b[NF * gn + f] - tv[f];
#pragma unroll
    for (int a = 0; a < NF; ++a) {
        T acc = T(0);
#pragma unroll
        for (int c = 0; c < NF; ++c)
            acc += (OP == OP_JTV ? Dn[c * NF + a] : Dn[a * NF + c]) * rr[c];
        x[NF * gn + a] += omega * acc;
    }
}

template <typename T, int OP>
__global__ __launch_bounds__(256) void k_combine_smooth(Geo g, const T *__restrict__ slots,
                                                        const uint8_t *__restrict__ nmask,
                                                        const T *__restrict__ t,
                                                        const T *__restrict__ D,
                                                        const T *__restrict__ b, T *x, T omega)
{
    combine_smooth_nodes<T, OP>(g, slots, nmask, t, D, b, x, omega, blockIdx.x);
}

// ---- design derivative: one output per element, no scatter ---------------------

__global__ __launch_bounds__(NTHR) void k_dRdgamma(Geo g, const double *__restrict__ x,
                                                   const double *__restrict__ lam,
                                                   const double *__restrict__ gamma,
                                                   const double *__restrict__ src,
                                                   const uint8_t *__restrict__ nmask,
                                                   double *__restrict__ gout)
{
    using T = double;
    constexpr bool UNR = Unroll<T>::value;
    __shared__ T sx[NF][BOXN];
    __shared__ T sl[NF][BOXN];
    const TileIdx t = tile_index(g);
    stage<T, 0, true>(g, t, x, lam, nmask, sx, sl, nullptr);
    __syncthreads();
    if (!t.valid) return;
    const EC<T> c = make_ec<T>(g);
    const int64_t e = (int64_t)t.i + (int64_t)g.nx * ((int64_t)t.j + (int64_t)g.ny * t.k);
    const double y = gamma[e];
    const T alpha = alpha_of(g, y), Kc = K_of(g, y), s = src[e];
    const T da = dalpha_of(g, y), dK = dK_of(g, y);
    T mu[3][8], mL[3][8], mp[8], mT[8], mP[8], mTh[8];
    T U2 = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            T xa = sx[i][t.nb[a]];
            U2 += xa * xa;
            mu[i][a] = xa;
            mL[i][a] = sl[i][t.nb[a]];
        }
        to_modal(mu[i], c);
        to_modal(mL[i], c);
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        mp[a] = sx[3][t.nb[a]];
        mT[a] = sx[4][t.nb[a]];
        mP[a] = sl[3][t.nb[a]];
        mTh[a] = sl[4][t.nb[a]];
    }
    to_modal(mp, c);
    to_modal(mT, c);
    to_modal(mP, c);
    to_modal(mTh, c);
    const T tau = rsqrt_t(U2 * c.inv16h2 + c.cvisc + alpha * alpha);
    const T tauT = rsqrt_t(U2 * c.inv16h2 + Kc * Kc * c.c16h4);
    const T dtau_da = -(tau * tau * tau) * alpha;                 // d tau / d alpha
    const T dtauT_dK = -(tauT * tauT * tauT) * Kc * c.c16h4;      // d tauT / d K
    T ga = 0, gk = 0;
    const T gs = c.gs;
#define FE_DG_GP(SG)                                                                          \
    {                                                                                        \
        T u[3], Gd[3][3], L[3], LG[3][3];                                                    \
        _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                      \
            eval_vg(SG, mu[i], gs, u[i], Gd[i][0], Gd[i][1], Gd[i][2]);                       \
            eval_vg(SG, mL[i], gs, L[i], LG[i][0], LG[i][1], LG[i][2]);                       \
        }                                                                                    \
        T gp[3], Tv, gT[3], gP[3], gTh[3];                                                   \
        eval_g(SG, mp, gs, gp[0], gp[1], gp[2]);                                              \
        eval_vg(SG, mT, gs, Tv, gT[0], gT[1], gT[2]);                                         \
        eval_g(SG, mP, gs, gP[0], gP[1], gP[2]);                                              \
        eval_g(SG, mTh, gs, gTh[0], gTh[1], gTh[2]);                                          \
        const T egv[3] = {c.eg0, c.eg1, c.eg2};                                              \
        _Pragma("unroll") for (int i = 0; i < 3; ++i) {                                      \
            T rM = u[0] * Gd[i][0] + u[1] * Gd[i][1] + u[2] * Gd[i][2] + gp[i]              \
                 + alpha * u[i] + c.B * egv[i] * Tv;                                         \
            T q = u[0] * LG[i][0] + u[1] * LG[i][1] + u[2] * LG[i][2] + gP[i];               \
            ga += L[i] * u[i] + dtau_da * q * rM + tau * q * u[i];                           \
        }                                                                                    \
        T rT = u[0] * gT[0] + u[1] * gT[1] + u[2] * gT[2] - s;                               \
        T uTh = u[0] * gTh[0] + u[1] * gTh[1] + u[2] * gTh[2];                               \
        gk += gTh[0] * gT[0] + gTh[1] * gT[1] + gTh[2] * gT[2] + dtauT_dK * uTh * rT;        \
    }
    FE_GAUSS_LOOP(UNR, T, FE_DG_GP)
#undef FE_DG_GP
    gout[e] = c.W * (da * ga + dK * gk);
}

// ---- nodal 5x5 diagonal blocks of J -----------------------------------------------

// Shape function of local node a and its physical gradient at Gauss point G.
template <typename T, typename SGT>
__device__ __forceinline__ void shape_at(const SGT &SG, int a, T h, T &N, T dN[3])
{
    const T q = (T)QG;
    const T sgv[3] = {T(SG.sx), T(SG.sy), T(SG.sz)};
    T f[3], sgn[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T sg = sgv[d] * q;
        sgn[d] = ((a >> d) & 1) ? T(1) : T(-1);
        f[d] = T(0.5) * (T(1) + sgn[d] * sg);
    }
    N = f[0] * f[1] * f[2];
    dN[0] = (sgn[0] / h) * f[1] * f[2];
    dN[1] = (sgn[1] / h) * f[0] * f[2];
    dN[2] = (sgn[2] / h) * f[0] * f[1];
}

// Corners per group of the block kernel, FP64 and FP32.  With the node box in
// the accumulators' LDS, one FP64 corner per group (252 registers) lets two
// waves share a SIMD; with 2 (322 registers, 1.5x faster than evaluating each
// corner's derivatives separately) only one fits (64^3 / 160x160x320, blocks
// and shared-node pass: 243 us / 6.15 ms with 1 corner, 297 us / 8.29 ms with 2,
// 285 us / 7.89 ms with 4).
#ifndef FE_BD_GROUP
#define FE_BD_GROUP 1
#endif
#ifndef FE_BD_GROUP32
#define FE_BD_GROUP32 2
#endif
template <typename T>
struct BdCfg;
template <>
struct BdCfg<double> {
    static constexpr int G = FE_BD_GROUP, WAVES = FE_BD_GROUP == 1 ? 2 : 1;
};
template <>
struct BdCfg<float> {
    static constexpr int G = FE_BD_GROUP32, WAVES = 2;
};

// State at one Gauss point: velocity, its gradient G[i][j] = d u_i / d x_j,
// the strong momentum residual and the temperature gradient and residual.
template <typename T>
struct BdState {
    T u[3], G[3][3], rM[3], gT[3], rT;
};

// Unscaled (without the Gauss weight W) contribution of one Gauss point to the
// nodal 5x5 block of corner a: row f, column k of
// sum_g W d R_{f,a} / d x_{k,a}, the directional derivative of the element
// residual (Galerkin + SUPG/PSPG with tau and tauT, and their variation with
// the element velocity) along the unit vector of DOF (a, k).  With N = N_a and
// d = grad N_a at the point, udN = u . d, and dtau_k = -tau^3 u_{a,k}/(16 h^2)
// (likewise dtauT_k), the terms are those of J v with v = N e_k:
//   velocity columns k < 3:
//     [i][k] = N (N + tau udN) G_ik + delta_ik ((udN + alpha N)(N + tau udN) + Pr |d|^2)
//              + Pr d_i d_k + rM_i (udN dtau_k + tau N d_k)
//     [3][k] = N d_k + dtau_k (d . rM) + tau (N (d . G_{.k}) + d_k (udN + alpha N))
//     [4][k] = N gT_k (N + tauT udN) + rT (udN dtauT_k + tauT N d_k)
//   pressure column: [i][3] = d_i (tau udN - N), [3][3] = tau |d|^2, [4][3] = 0
//   temperature column: [i][4] = B eg_i N (N + tau udN), [3][4] = tau B N (eg . d),
//     [4][4] = N udN + K |d|^2 + tauT udN^2.
template <typename T>
__device__ __forceinline__ void bd_corner(const EC<T> &c, const BdState<T> &st, T N, const T dN[3],
                                          const T ua[3], T alpha, T Kc, T tau, T tauT, T blk[25])
{
    const T udN = st.u[0] * dN[0] + st.u[1] * dN[1] + st.u[2] * dN[2];
    const T dd = dN[0] * dN[0] + dN[1] * dN[1] + dN[2] * dN[2];
    const T Nt = N + tau * udN, NtT = N + tauT * udN;
    const T uaN = udN + alpha * N;
    const T c1 = N * Nt;
    const T c2 = uaN * Nt + c.Pr * dd;
    const T t3 = tau * tau * tau * c.inv16h2, t3T = tauT * tauT * tauT * c.inv16h2;
    const T drM = dN[0] * st.rM[0] + dN[1] * st.rM[1] + dN[2] * st.rM[2];
    const T egv[3] = {c.eg0, c.eg1, c.eg2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T dtk = -t3 * ua[k], dtTk = -t3T * ua[k];
        const T ek = udN * dtk + tau * N * dN[k];
        const T dGk = dN[0] * st.G[0][k] + dN[1] * st.G[1][k] + dN[2] * st.G[2][k];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T v = c1 * st.G[i][k] + c.Pr * dN[i] * dN[k] + st.rM[i] * ek;
            if (i == k) v += c2;
            blk[i * NF + k] += v;
        }
        blk[3 * NF + k] += N * dN[k] + dtk * drM + tau * (N * dGk + dN[k] * uaN);
        blk[4 * NF + k] += N * st.gT[k] * NtT + st.rT * (udN * dtTk + tauT * N * dN[k]);
    }
    const T pq = tau * udN - N, bN = c.B * N * Nt;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        blk[i * NF + 3] += dN[i] * pq;
        blk[i * NF + 4] += egv[i] * bN;
    }
    blk[3 * NF + 3] += tau * dd;
    blk[3 * NF + 4] += tau * c.B * N * (egv[0] * dN[0] + egv[1] * dN[1] + egv[2] * dN[2]);
    blk[4 * NF + 4] += N * udN + Kc * dd + tauT * udN * udN;
}

// Nodal 5x5 diagonal blocks of J at state x in the arithmetic of T (FP32 for
// the mixed-precision preconditioner, whose smoother only uses FP32 blocks).
template <typename T>
__global__ __launch_bounds__(NTHR, BdCfg<T>::WAVES) void k_blockdiag(Geo g, const T *__restrict__ x,
                                                    const double *__restrict__ gamma,
                                                    const double *__restrict__ src,
                                                    const uint8_t *__restrict__ nmask,
                                                    T *__restrict__ D,
                                                    T *__restrict__ slots)
{
    // 25 accumulators per box node (81,000 B); the staged node box lives in the
    // same array until the element state is in registers, so that two
    // workgroups fit in a CU's LDS
    __shared__ T so[25 * BOXN];
    T(*sx)[BOXN] = reinterpret_cast<T(*)[BOXN]>(so);
    const TileIdx t = tile_index(g);
    stage<T, 0, false>(g, t, x, (const T *)nullptr, nmask, sx, nullptr, nullptr);
    __syncthreads();
    const EC<T> c = make_ec<T>(g);
    T alpha = 0, Kc = 1, s = 0, tau = 0, tauT = 0;
    T mu[3][8], mp[8], mT[8];
    if (t.valid) {
        const int64_t e = (int64_t)t.i + (int64_t)g.nx * ((int64_t)t.j + (int64_t)g.ny * t.k);
        const double y = gamma[e];
        alpha = (T)alpha_of(g, y);
        Kc = (T)K_of(g, y);
        s = (T)src[e];
        T U2 = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                T xa = sx[i][t.nb[a]];
                U2 += xa * xa;
                mu[i][a] = xa;
            }
            to_modal(mu[i], c);
        }
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            mp[a] = sx[3][t.nb[a]];
            mT[a] = sx[4][t.nb[a]];
        }
        to_modal(mp, c);
        to_modal(mT, c);
        tau = rsqrt_t(U2 * c.inv16h2 + c.cvisc + alpha * alpha);
        tauT = rsqrt_t(U2 * c.inv16h2 + Kc * Kc * c.c16h4);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 25 * BOXN; idx += NTHR) so[idx] = T(0);
    __syncthreads();
    const T h = (T)g.h;
    // Corners in groups of BDG: the state at each Gauss point is evaluated once
    // per group (8 / BDG times per element instead of once per corner), and
    // each corner's block is the closed form of the directional derivatives
    // along the five unit vectors of that node (see bd_corner).  The corners'
    // nodal velocities are read from x (the staged copy is overwritten), one
    // group ahead.  The accumulation keeps the corner order of the sub-steps.
    constexpr int BDG = BdCfg<T>::G;
    auto corner_u = [&](int a, T u[3]) {
        const int64_t n = gnode(g, t.i + (a & 1), t.j + ((a >> 1) & 1), t.k + (a >> 2));
#pragma unroll
        for (int k = 0; k < 3; ++k) u[k] = x[NF * n + k];
    };
    T un[BDG][3];
    if (t.valid) {
#pragma unroll
        for (int cc = 0; cc < BDG; ++cc) corner_u(cc, un[cc]);
    }
#pragma unroll 1
    for (int grp = 0; grp < 8 / BDG; ++grp) {
        T blk[BDG][25];
#pragma unroll
        for (int cc = 0; cc < BDG; ++cc)
#pragma unroll
            for (int q = 0; q < 25; ++q) blk[cc][q] = T(0);
        if (t.valid) {
            T ua[BDG][3];
#pragma unroll
            for (int cc = 0; cc < BDG; ++cc)
#pragma unroll
                for (int k = 0; k < 3; ++k) ua[cc][k] = un[cc][k];
            if (grp + 1 < 8 / BDG) {
#pragma unroll
                for (int cc = 0; cc < BDG; ++cc) corner_u(BDG * (grp + 1) + cc, un[cc]);
            }
#define FE_BD2_GP(SG)                                                                         \
    {                                                                                        \
        BdState<T> st;                                                                       \
        _Pragma("unroll") for (int i = 0; i < 3; ++i)                                        \
            eval_vg(SG, mu[i], c.gs, st.u[i], st.G[i][0], st.G[i][1], st.G[i][2]);           \
        T gp[3], Tv;                                                                         \
        eval_g(SG, mp, c.gs, gp[0], gp[1], gp[2]);                                            \
        eval_vg(SG, mT, c.gs, Tv, st.gT[0], st.gT[1], st.gT[2]);                              \
        const T egv[3] = {c.eg0, c.eg1, c.eg2};                                              \
        _Pragma("unroll") for (int i = 0; i < 3; ++i)                                        \
            st.rM[i] = st.u[0] * st.G[i][0] + st.u[1] * st.G[i][1] + st.u[2] * st.G[i][2]   \
                     + gp[i] + alpha * st.u[i] + c.B * egv[i] * Tv;                          \
        st.rT = st.u[0] * st.gT[0] + st.u[1] * st.gT[1] + st.u[2] * st.gT[2] - s;            \
        _Pragma("unroll") for (int cc = 0; cc < BDG; ++cc) {                                 \
            T N, dN[3];                                                                      \
            shape_at(SG, BDG * grp + cc, h, N, dN);                                          \
            bd_corner(c, st, N, dN, ua[cc], alpha, Kc, tau, tauT, blk[cc]);                   \
        }                                                                                    \
    }
            FE_GAUSS_LOOP(false, T, FE_BD2_GP)
#undef FE_BD2_GP
        }
#pragma unroll
        for (int cc = 0; cc < BDG; ++cc) {
            if (t.valid) {
#pragma unroll
                for (int q = 0; q < 25; ++q) so[q * BOXN + t.nb[BDG * grp + cc]] += c.W * blk[cc][q];
            }
            __syncthreads();
        }
    }
    // write-out, one thread per (node, entry): consecutive threads store
    // consecutive entries of a node, and consecutive nodes of a box row are
    // consecutive in D and in the slots
    const int tx0 = t.btx * TX, ty0 = t.bty * TY, tz0 = t.btz * TZ;
    for (int idx = threadIdx.x; idx < 25 * BOXN; idx += NTHR) {
        const int nb = idx / 25, q = idx - 25 * nb;
        const int lx = nb % BX, r = nb / BX, ly = r % BY, lz = r / BY;
        const int I = tx0 + lx, J = ty0 + ly, K = tz0 + lz;
        if (I > g.nx || J > g.ny || K > g.nz) continue;
        const bool sh = shared_dir(lx, I, g.nx, TX) || shared_dir(ly, J, g.ny, TY) ||
                        shared_dir(lz, K, g.nz, TZ);
        const T val = so[q * BOXN + nb];
        if (sh) {
            slots[((int64_t)t.tile * BOXN + nb) * 25 + q] = val;
        } else {
            const int64_t gn = gnode(g, I, J, K);
            const uint8_t m = nmask[gn];
            const int f = q / NF, f2 = q - NF * f;
            D[gn * 25 + q] = (((m >> f) & 1) || ((m >> f2) & 1)) ? ((f == f2) ? T(1) : T(0)) : val;
        }
    }
}

// ---- batched launches: the kernels above over a table of problems -------------

template <typename Tin, typename Tout>
__global__ __launch_bounds__(NTHR) void kb_elem_jv(const BElem<Tin, Tout> *__restrict__ tab,
                                                   const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BElem<Tin, Tout> &a = tab[e];
    const int b0 = off[e];
    elem_tile<Tin, Tout, OP_JV>(a.g, a.x, a.v, a.gamma, a.s, a.nmask, a.out, a.slots,
                                (int)blockIdx.x - b0, off[e + 1] - b0);
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void kb_combine_jv(const BElem<Tin, Tout> *__restrict__ tab,
                                                     const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BElem<Tin, Tout> &a = tab[e];
    combine_nodes<Tin, Tout, NF, OP_JV>(a.g, a.slots, a.nmask, a.v, a.out,
                                        blockIdx.x - (unsigned)off[e]);
}

template <typename T>
__global__ __launch_bounds__(NTHR) void kb_elem_smooth(const BElemSmooth<T> *__restrict__ tab,
                                                       const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BElemSmooth<T> &a = tab[e];
    const int b0 = off[e];
    elem_tile<T, T, OP_JV>(a.g, a.xs, (const T *)a.x, a.gamma, a.s, a.nmask, a.t, a.slots,
                           (int)blockIdx.x - b0, off[e + 1] - b0);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_combine_smooth(const BElemSmooth<T> *__restrict__ tab,
                                                         const int *__restrict__ off, int n)
{
    const int e = batch_entry(off, n);
    const BElemSmooth<T> &a = tab[e];
    combine_smooth_nodes<T, OP_JV>(a.g, a.slots, a.nmask, a.t, a.D, a.b, a.x, a.omega,
                                   blockIdx.x - (unsigned)off[e]);
}

}  // namespace

// ---- assembled operator of a small grid (coarsest multigrid level) -----------------

// Element Jacobians: thread (e, c) evaluates J_e e_c, the 40 element rows for the
// unit direction on local DOF c = 8 f + a (corner a, field f); a prescribed DOF
// gives a zero direction, as in fe_jvp.  Je is [element][row][column], 40 x 40.
__global__ __launch_bounds__(64) void k_elem_jac(Geo g, const double *__restrict__ x,
                                                 const double *__restrict__ gamma,
                                                 const double *__restrict__ src,
                                                 const uint8_t *__restrict__ nmask,
                                                 double *__restrict__ Je)
{
    const int64_t ne = n_elem(g);
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= ne * 40) return;
    const int64_t e = tid / 40;
    const int col = (int)(tid - e * 40);
    const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((int64_t)g.nx * g.ny));
    int64_t nd[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) nd[a] = gnode(g, i + (a & 1), j + ((a >> 1) & 1), k + (a >> 2));
    const int fc = col >> 3, ac = col & 7;
    const double one = ((nmask[nd[ac]] >> fc) & 1) ? 0.0 : 1.0;
    const EC<double> c = make_ec<double>(g);
    const double y = gamma[e];
    const double alpha = alpha_of(g, y), Kc = K_of(g, y), s = src[e];
    double R[NF][8];
    elem_jv<double, false>(
        c, [&](int f, int a) { return x[NF * nd[a] + f]; },
        [&](int f, int a) { return (8 * f + a == col) ? one : 0.0; }, alpha, Kc, s, R);
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int a = 0; a < 8; ++a) Je[(e * 40 + 8 * f + a) * 40 + col] = R[f][a];
}

// The 135 probing products J p_q of a small grid from its element Jacobians:
// p_q is the sum of the unit vectors of field f (q = 5 col + f) on the nodes of
// colour col = (I mod 3) + 3 (J mod 3) + 9 (K mod 3).  Every element has at most
// one corner of a colour, so row (N, g) of J p_q sums one element entry per
// element around N, in increasing element order.  Prescribed rows are identity rows.
__global__ __launch_bounds__(256) void k_probe_from_jac(Geo g, const double *__restrict__ Je,
                                                        const uint8_t *__restrict__ nmask,
                                                        double *__restrict__ probe_out)
{
    const int64_t nn = n_nodes(g), ndof = NF * nn;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= 135 * ndof) return;
    const int q = (int)(tid / ndof);
    const int64_t row = tid - (int64_t)q * ndof;
    const int64_t N = row / NF;
    const int gr = (int)(row - N * NF);
    const int colr = q / NF, f = q - colr * NF;
    const int I = (int)(N % (g.nx + 1)), J = (int)((N / (g.nx + 1)) % (g.ny + 1)),
              K = (int)(N / ((int64_t)(g.nx + 1) * (g.ny + 1)));
    const int colN = (I % 3) + 3 * (J % 3) + 9 * (K % 3);
    if ((nmask[N] >> gr) & 1) {
        probe_out[tid] = (colN == colr && f == gr) ? 1.0 : 0.0;
        return;
    }
    double acc = 0.0;
    for (int dz = -1; dz <= 0; ++dz)
        for (int dy = -1; dy <= 0; ++dy)
            for (int dx = -1; dx <= 0; ++dx) {
                const int ei = I + dx, ej = J + dy, ek = K + dz;
                if (ei < 0 || ej < 0 || ek < 0 || ei >= g.nx || ej >= g.ny || ek >= g.nz) continue;
                const int64_t e = ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek);
                const int aN = (-dx) | ((-dy) << 1) | ((-dz) << 2);
                for (int b = 0; b < 8; ++b) {
                    const int mi = ei + (b & 1), mj = ej + ((b >> 1) & 1), mk = ek + (b >> 2);
                    if ((mi % 3) + 3 * (mj % 3) + 9 * (mk % 3) != colr) continue;
                    acc += Je[(e * 40 + 8 * gr + aN) * 40 + 8 * f + b];
                    break;
                }
            }
    probe_out[tid] = acc;
}

// The assembled operator of a small grid as a 27-point block stencil, from its
// element Jacobians: S[((d 5 + g) 5 + f) nn + N] is entry (N g, M f) with
// M = N + (dx, dy, dz), d = (dx + 1) + 3 (dy + 1) + 9 (dz + 1).  The entry sums
// one element entry per element around N that also holds M, in increasing
// element order (the order of the probing products above).  Prescribed rows
// are identity rows; prescribed columns are zero in Je already; neighbours
// outside the grid give zero entries.
__global__ __launch_bounds__(256) void k_stencil_from_jac(Geo g, const double *__restrict__ Je,
                                                          const uint8_t *__restrict__ nmask,
                                                          double *__restrict__ S)
{
    const int64_t nn = n_nodes(g);
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= 675 * nn) return;
    const int q = (int)(tid / nn);
    const int64_t N = tid - (int64_t)q * nn;
    const int d = q / 25, gr = (q / NF) % NF, f = q % NF;
    const int ddx = d % 3 - 1, ddy = (d / 3) % 3 - 1, ddz = d / 9 - 1;
    const int I = (int)(N % (g.nx + 1)), J = (int)((N / (g.nx + 1)) % (g.ny + 1)),
              K = (int)(N / ((int64_t)(g.nx + 1) * (g.ny + 1)));
    if ((nmask[N] >> gr) & 1) {
        S[tid] = (d == 13 && f == gr) ? 1.0 : 0.0;
        return;
    }
    double acc = 0.0;
    for (int dz = -1; dz <= 0; ++dz)
        for (int dy = -1; dy <= 0; ++dy)
            for (int dx = -1; dx <= 0; ++dx) {
                const int ei = I + dx, ej = J + dy, ek = K + dz;
                if (ei < 0 || ej < 0 || ek < 0 || ei >= g.nx || ej >= g.ny || ek >= g.nz) continue;
                // corners of N and of M in this element
                const int bx = -dx + ddx, by = -dy + ddy, bz = -dz + ddz;
                if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
                const int64_t e = ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek);
                const int aN = (-dx) | ((-dy) << 1) | ((-dz) << 2);
                const int b = bx | (by << 1) | (bz << 2);
                acc += Je[(e * 40 + 8 * gr + aN) * 40 + 8 * f + b];
            }
    S[tid] = acc;
}

// ---- launchers ----------------------------------------------------------------------

template <typename Tin, typename Tout>
hipError_t launch_elem(ElemOp op, const Geo &g, const Tin *x, const Tin *v, const double *gamma,
                       const double *s, const uint8_t *nmask, Tout *out, Tout *slots,
                       hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    const dim3 grid((unsigned)n_tiles(g)), block(NTHR);
    const int64_t nn = n_nodes(g);
    const dim3 cgrid((unsigned)((nn + 255) / 256)), cblock(256);
    switch (op) {
    case OP_RES:
        hipLaunchKernelGGL((k_elem<Tin, Tout, OP_RES>), grid, block, 0, st, g, x, v, gamma, s,
                           nmask, out, slots);
        hipLaunchKernelGGL((k_combine<Tin, Tout, NF, OP_RES>), cgrid, cblock, 0, st, g,
                           (const Tout *)slots, nmask, v, out);
        break;
    case OP_JV:
        if (ev0) {
            const hipError_t e = hipEventRecord(ev0, st);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((k_elem<Tin, Tout, OP_JV>), grid, block, 0, st, g, x, v, gamma, s,
                           nmask, out, slots);
        if (ev1) {
            const hipError_t e = hipEventRecord(ev1, st);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((k_combine<Tin, Tout, NF, OP_JV>), cgrid, cblock, 0, st, g,
                           (const Tout *)slots, nmask, v, out);
        break;
    case OP_JTV:
        hipLaunchKernelGGL((k_elem<Tin, Tout, OP_JTV>), grid, block, 0, st, g, x, v, gamma, s,
                           nmask, out, slots);
        hipLaunchKernelGGL((k_combine<Tin, Tout, NF, OP_JTV>), cgrid, cblock, 0, st, g,
                           (const Tout *)slots, nmask, v, out);
        break;
    }
    return hipGetLastError();
}

template hipError_t launch_elem<double, double>(ElemOp, const Geo &, const double *, const double *,
                                                const double *, const double *, const uint8_t *,
                                                double *, double *, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_elem<float, float>(ElemOp, const Geo &, const float *, const float *,
                                              const double *, const double *, const uint8_t *,
                                              float *, float *, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_elem<float, double>(ElemOp, const Geo &, const float *, const float *,
                                               const double *, const double *, const uint8_t *,
                                               double *, double *, hipStream_t, hipEvent_t, hipEvent_t);

hipError_t launch_elem_dir32(ElemOp op, const Geo &g, const double *x, const float *v,
                             const double *gamma, const double *s, const uint8_t *nmask,
                             double *out, double *slots, hipStream_t st)
{
    const dim3 grid((unsigned)n_tiles(g)), block(NTHR);
    const int64_t nn = n_nodes(g);
    const dim3 cgrid((unsigned)((nn + 255) / 256)), cblock(256);
    if (op == OP_JV) {
        hipLaunchKernelGGL((k_elem_dir32<OP_JV>), grid, block, 0, st, g, x, v, gamma, s, nmask,
                           out, slots);
        hipLaunchKernelGGL((k_combine<float, double, NF, OP_JV>), cgrid, cblock, 0, st, g,
                           (const double *)slots, nmask, v, out);
    } else if (op == OP_JTV) {
        hipLaunchKernelGGL((k_elem_dir32<OP_JTV>), grid, block, 0, st, g, x, v, gamma, s, nmask,
                           out, slots);
        hipLaunchKernelGGL((k_combine<float, double, NF, OP_JTV>), cgrid, cblock, 0, st, g,
                           (const double *)slots, nmask, v, out);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dRdgamma(const Geo &g, const double *x, const double *lam, const double *gamma,
                           const double *s, const uint8_t *nmask, double *gout, hipStream_t st)
{
    hipLaunchKernelGGL(k_dRdgamma, dim3((unsigned)n_tiles(g)), dim3(NTHR), 0, st, g, x, lam, gamma,
                       s, nmask, gout);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_blockdiag(const Geo &g, const T *x, const double *gamma, const double *s,
                            const uint8_t *nmask, T *D, T *slots, hipStream_t st)
{
    hipLaunchKernelGGL(k_blockdiag<T>, dim3((unsigned)n_tiles(g)), dim3(NTHR), 0, st, g, x, gamma,
                       s, nmask, D, slots);
    const int64_t nn = n_nodes(g);
    hipLaunchKernelGGL((k_combine<T, T, 25, OP_RES>), dim3((unsigned)((nn + 255) / 256)),
                       dim3(256), 0, st, g, (const T *)slots, nmask, (const T *)nullptr, D);
    return hipGetLastError();
}
template hipError_t launch_blockdiag<double>(const Geo &, const double *, const double *,
                                             const double *, const uint8_t *, double *, double *,
                                             hipStream_t);
template hipError_t launch_blockdiag<float>(const Geo &, const float *, const double *,
                                            const double *, const uint8_t *, float *, float *,
                                            hipStream_t);

template <typename T>
hipError_t launch_elem_smooth(bool tr, const Geo &g, const T *xs, T *x, const double *gamma,
                              const double *s, const uint8_t *nmask, T *t, T *slots, const T *D,
                              const T *b, T omega, hipStream_t st)
{
    const dim3 grid((unsigned)n_tiles(g)), block(NTHR);
    const int64_t nn = n_nodes(g);
    const dim3 cgrid((unsigned)((nn + 255) / 256)), cblock(256);
    if (tr) {
        hipLaunchKernelGGL((k_elem<T, T, OP_JTV>), grid, block, 0, st, g, xs, (const T *)x, gamma,
                           s, nmask, t, slots);
        hipLaunchKernelGGL((k_combine_smooth<T, OP_JTV>), cgrid, cblock, 0, st, g,
                           (const T *)slots, nmask, (const T *)t, D, b, x, omega);
    } else {
        hipLaunchKernelGGL((k_elem<T, T, OP_JV>), grid, block, 0, st, g, xs, (const T *)x, gamma, s,
                           nmask, t, slots);
        hipLaunchKernelGGL((k_combine_smooth<T, OP_JV>), cgrid, cblock, 0, st, g,
                           (const T *)slots, nmask, (const T *)t, D, b, x, omega);
    }
    return hipGetLastError();
}
template hipError_t launch_elem_smooth<double>(bool, const Geo &, const double *, double *,
                                               const double *, const double *, const uint8_t *,
                                               double *, double *, const double *, const double *,
                                               double, hipStream_t);
template hipError_t launch_elem_smooth<float>(bool, const Geo &, const float *, float *,
                                              const double *, const double *, const uint8_t *,
                                              float *, float *, const float *, const float *, float,
                                              hipStream_t);

hipError_t launch_stencil_assemble(const Geo &g, const double *x, const double *gamma,
                                   const double *s, const uint8_t *nmask, double *Je, double *S,
                                   hipStream_t st)
{
    const int64_t ne = n_elem(g), nn = n_nodes(g);
    hipLaunchKernelGGL(k_elem_jac, dim3((unsigned)((ne * 40 + 63) / 64)), dim3(64), 0, st, g, x,
                       gamma, s, nmask, Je);
    hipLaunchKernelGGL(k_stencil_from_jac, dim3((unsigned)((675 * nn + 255) / 256)), dim3(256), 0,
                       st, g, (const double *)Je, nmask, S);
    return hipGetLastError();
}

hipError_t launch_probe_products(const Geo &g, const double *x, const double *gamma,
                                 const double *s, const uint8_t *nmask, double *Je,
                                 double *probe_out, hipStream_t st)
{
    const int64_t ne = n_elem(g), ndof = NF * n_nodes(g);
    hipLaunchKernelGGL(k_elem_jac, dim3((unsigned)((ne * 40 + 63) / 64)), dim3(64), 0, st, g, x,
                       gamma, s, nmask, Je);
    hipLaunchKernelGGL(k_probe_from_jac, dim3((unsigned)((135 * ndof + 255) / 256)), dim3(256), 0,
                       st, g, (const double *)Je, nmask, probe_out);
    return hipGetLastError();
}

// ---- batched launchers ---------------------------------------------------------------

template <typename Tin, typename Tout>
hipError_t blaunch_elem_jv(const BLaunch &L, hipStream_t st)
{
    if (L.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((kb_elem_jv<Tin, Tout>), dim3((unsigned)L.blocks), dim3(NTHR), 0, st,
                       (const BElem<Tin, Tout> *)L.tab, L.off, L.n);
    return hipGetLastError();
}

template <typename Tin, typename Tout>
hipError_t blaunch_combine_jv(const BLaunch &L, hipStream_t st)
{
    if (L.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((kb_combine_jv<Tin, Tout>), dim3((unsigned)L.blocks), dim3(256), 0, st,
                       (const BElem<Tin, Tout> *)L.tab, L.off, L.n);
    return hipGetLastError();
}

template <typename T>
hipError_t blaunch_elem_smooth_pass(const BLaunch &L, hipStream_t st)
{
    if (L.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((kb_elem_smooth<T>), dim3((unsigned)L.blocks), dim3(NTHR), 0, st,
                       (const BElemSmooth<T> *)L.tab, L.off, L.n);
    return hipGetLastError();
}

template <typename T>
hipError_t blaunch_combine_smooth(const BLaunch &L, hipStream_t st)
{
    if (L.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((kb_combine_smooth<T>), dim3((unsigned)L.blocks), dim3(256), 0, st,
                       (const BElemSmooth<T> *)L.tab, L.off, L.n);
    return hipGetLastError();
}

template hipError_t blaunch_elem_jv<double, double>(const BLaunch &, hipStream_t);
template hipError_t blaunch_elem_jv<float, double>(const BLaunch &, hipStream_t);
template hipError_t blaunch_elem_jv<float, float>(const BLaunch &, hipStream_t);
template hipError_t blaunch_combine_jv<double, double>(const BLaunch &, hipStream_t);
template hipError_t blaunch_combine_jv<float, double>(const BLaunch &, hipStream_t);
template hipError_t blaunch_combine_jv<float, float>(const BLaunch &, hipStream_t);
template hipError_t blaunch_elem_smooth_pass<double>(const BLaunch &, hipStream_t);
template hipError_t blaunch_elem_smooth_pass<float>(const BLaunch &, hipStream_t);
template hipError_t blaunch_combine_smooth<double>(const BLaunch &, hipStream_t);
template hipError_t blaunch_combine_smooth<float>(const BLaunch &, hipStream_t);

}  // namespace fe
