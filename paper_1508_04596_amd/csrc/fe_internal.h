// Internal declarations of the HIP state-solver library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstdint>
#include <string>
#include <vector>

#include "fe.h"

namespace fe {

constexpr int NF = 5;  // unknowns per node: u, v, w, p, T

// Element tile processed by one workgroup: TX*TY*TZ elements, one per thread.
#ifndef FE_TILE_X
#define FE_TILE_X 8
#endif
#ifndef FE_TILE_Y
#define FE_TILE_Y 8
#endif
#ifndef FE_TILE_Z
#define FE_TILE_Z 4
#endif
constexpr int TX = FE_TILE_X, TY = FE_TILE_Y, TZ = FE_TILE_Z;
constexpr int NTHR = TX * TY * TZ;  // 256 threads = 4 wave64
constexpr int BX = TX + 1, BY = TY + 1, BZ = TZ + 1;
constexpr int BOXN = BX * BY * BZ;  // nodes of the tile's node box (405)

// Grid geometry and physical constants, passed by value to every element kernel.
struct Geo {
    int nx, ny, nz;     // elements
    int ntx, nty, ntz;  // tiles
    double h, Pr, B;    // B = Gr * Pr^2 (buoyancy coefficient)
    double eg[3];
    double Ck, qf, amax, qa;
    // derived per-launch constants (host-computed)
    double W;        // (h/2)^3
    double gs;       // 2/(h/sqrt(3))
    double igs;      // 1/gs
    double inv16h2;  // 1/(16 h^2)
    double cvisc;    // 16 Pr^2 / h^4
    double c16h4;    // 16 / h^4
};

Geo make_geo(const fe_grid &g, const fe_phys &ph);

__host__ __device__ inline int64_t n_nodes(const Geo &g)
{
    return (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
}
__host__ __device__ inline int64_t n_elem(const Geo &g) { return (int64_t)g.nx * g.ny * g.nz; }
inline int64_t n_tiles(const Geo &g) { return (int64_t)g.ntx * g.nty * g.ntz; }

// The nodal 5x5 blocks ([node][25], row-major) of the 256 consecutive nodes
// n0 .. n0 + 255 copied to LDS with coalesced loads, for kernels that run one
// thread per node: read directly, neighbouring lanes would fetch values 200 B
// apart, 25 scattered requests per wave where 25 contiguous ones suffice.
// Every thread of the 256-thread workgroup must call it (it synchronises the
// workgroup).  Entries past node nn - 1 hold copies of the last block.
// Returns this thread's block.
template <typename T>
__device__ __forceinline__ const T *stage_blocks256(const T *__restrict__ D, int64_t n0, int64_t nn,
                                                    T *sD)
{
    const int64_t left = nn - n0;
    const int cnt = (int)(left < 256 ? left : 256) * 25;
    const T *src = D + n0 * 25;
    T v[25];
#pragma unroll
    for (int k = 0; k < 25; ++k) {
        const int q = (int)threadIdx.x + 256 * k;
        v[k] = src[q < cnt ? q : cnt - 1];
    }
#pragma unroll
    for (int k = 0; k < 25; ++k) sD[threadIdx.x + 256 * k] = v[k];
    __syncthreads();
    return sD + threadIdx.x * 25;
}

// Which element operator a tile kernel evaluates.
enum ElemOp { OP_RES = 0, OP_JV = 1, OP_JTV = 2 };

// ---- element kernel launchers (fe_elem.hip) --------------------------------
// x, v: node vectors of type Tin; out: node vector of type Tout; nmask: per
// node bit mask (bit f set = DOF f prescribed); slots: tile-face partial sums,
// n_tiles * BOXN * 5 values of Tout.
// ev0/ev1 (optional): recorded on st right before and right after the J v
// element-pass kernel.
template <typename Tin, typename Tout>
hipError_t launch_elem(ElemOp op, const Geo &g, const Tin *x, const Tin *v, const double *gamma,
                       const double *s, const uint8_t *nmask, Tout *out, Tout *slots,
                       hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_dRdgamma(const Geo &g, const double *x, const double *lam, const double *gamma,
                           const double *s, const uint8_t *nmask, double *gout, hipStream_t st);
// J v (OP_JV) or J^T w (OP_JTV) in FP64 at an FP64 state x with the direction
// stored in FP32 (each value widened as it is staged; the masked entries of the
// output copy it): the operator of a solve whose preconditioner returns FP32
// vectors, without a separate widening pass.
hipError_t launch_elem_dir32(ElemOp op, const Geo &g, const double *x, const float *v,
                             const double *gamma, const double *s, const uint8_t *nmask,
                             double *out, double *slots, hipStream_t st);
// One smoother sweep with the operator fused: x += omega D^{-1} (b - J x) (J^T
// and D^{-T} when tr), J at state xs; t (node vector) and slots are work space.
template <typename T>
hipError_t launch_elem_smooth(bool tr, const Geo &g, const T *xs, T *x, const double *gamma,
                              const double *s, const uint8_t *nmask, T *t, T *slots, const T *D,
                              const T *b, T omega, hipStream_t st);
// Element Jacobians of grid g into Je (1600 per element), then its 27-point block
// stencil S (675 per node, [offset][row field][column field][node]).
hipError_t launch_stencil_assemble(const Geo &g, const double *x, const double *gamma,
                                   const double *s, const uint8_t *nmask, double *Je, double *S,
                                   hipStream_t st);
// The 135 colour-by-field probing products J p_q of a small grid, from element
// Jacobians (Je: n_elem * 1600 doubles of work space; probe_out: 135 * n_dof,
// product q at offset q * n_dof).
hipError_t launch_probe_products(const Geo &g, const double *x, const double *gamma,
                                 const double *s, const uint8_t *nmask, double *Je,
                                 double *probe_out, hipStream_t st);
// Raw nodal 5x5 diagonal blocks of J (row-major [n][25]) in the arithmetic of T,
// masked rows/cols set to the identity; slots must hold n_tiles * BOXN * 25 T.
template <typename T>
hipError_t launch_blockdiag(const Geo &g, const T *x, const double *gamma, const double *s,
                            const uint8_t *nmask, T *D, T *slots, hipStream_t st);

// ---- vector kernels (fe_vec.hip) ------------------------------------------
constexpr int RED_BLOCKS = 1024;  // partial sums per reduction (fixed => deterministic)
constexpr int RED_THREADS = 256;

hipError_t launch_node_mask(const uint8_t *dof_mask, uint8_t *nmask, int64_t nn, hipStream_t st);
// Invert 5x5 blocks in place (FP64) and optionally write an FP32 copy.
hipError_t launch_invert_blocks(double *D, float *D32, int64_t nn, hipStream_t st);
// In-place FP32 inverse of FP32 blocks (mixed-precision preconditioner set-up).
hipError_t launch_invert_blocks32(float *D32, int64_t nn, hipStream_t st);
// z = D v per node (D row-major 5x5); Tin/Tout/Tm = vector, output, matrix types;
// the transposed variant applies D^T.
template <typename Tm, typename Tin, typename Tout>
hipError_t launch_block_apply(const Tm *D, const Tin *v, Tout *z, int64_t nn, bool transpose,
                              const double *scale_dev, hipStream_t st);
// out[j] = sum_{b < nparts} partial[j*RED_BLOCKS + b] (+ add[j] if add != NULL),
// j < k, summed in a fixed order; if sqrt_last, out[k-1] = sqrt(out[k-1]).
hipError_t launch_reduce(const double *partial, int k, double *out, const double *add,
                         bool sqrt_last, hipStream_t st, int nparts = RED_BLOCKS);
// Workgroups (and partials per sum) of the Krylov vectors' reductions over n
// entries: at least two entries per thread, at most RED_BLOCKS (reached from
// n = 512 RED_BLOCKS on); short vectors thus avoid a grid of mostly idle
// workgroups.  The partition depends on n only, so the sums are deterministic.
inline int red_blocks(int64_t n)
{
    return (int)std::min<int64_t>(RED_BLOCKS, std::max<int64_t>(1, (n + 511) / 512));
}
hipError_t launch_norm2_partial(const double *a, int64_t n, double *partial, hipStream_t st);
// Columns of the reduction buffer `partial` (RED_BLOCKS partials each): the
// dot pass of a Gram-Schmidt step with J <= 63 final basis vectors fills 2J + 3.
constexpr int PARTIAL_COLS = 130;
// One FGMRES Arnoldi step's orthogonalisation by classical Gram-Schmidt with a
// delayed second projection (V of leading dimension ld: final basis vectors
// in columns 0 .. J-1, the scaled once-projected candidate in column J, the
// new Krylov vector w in column J + 1).  One pass reads the basis for all dot
// products, one pass updates: column J becomes the basis vector q_J (the
// candidate projected a second time and normalised), column J + 1 the next
// candidate (w projected once against q_0 .. q_J, divided by |w|).  hb (device)
// receives s_i = <q_i, c> at i < J, a = <c, c> at J, p_i = <q_i, w> at J + 1 + i,
// t = <c, w> at 2J + 1, e = <w, w> at 2J + 2, sigma = |c - sum s_i q_i|, the
// coefficient h = <q_J, w> and omega = |w| at 2J + 3 .. 2J + 5 and the squared
// norm of the next candidate at 2J + 8 (sigma = 0: nothing left of the
// candidate, q_J = 0).  0 <= J <= 63.
hipError_t launch_dgs_step(double *V, int64_t ld, int J, int64_t n, double *hb, double *partial,
                           hipStream_t st);
// The candidate's dot products alone (no new Krylov vector; it finishes the
// last Hessenberg column of a cycle): hb[i] = <q_i, c> for i < J, hb[J] = <c, c>.
// 1 <= J <= 64.
hipError_t launch_dgs_final(const double *V, int64_t ld, int J, int64_t n, double *hb,
                            double *partial, hipStream_t st);
// Givens rotations of the FGMRES least-squares problem (host): column c of H
// (m columns, row-major (m + 1) x m, entries 0 .. c+1 set) gets the rotations
// 0 .. c-1, defines rotation c and advances g; returns the residual estimate
// |g[c+1]|.  givens_estimate: the estimate that column c with entries
// col[0 .. c+1] would give, nothing changed.
double givens_column(std::vector<double> &H, int m, int c, std::vector<double> &cs,
                     std::vector<double> &sn, std::vector<double> &g);
double givens_estimate(const std::vector<double> &col, int c, const std::vector<double> &cs,
                       const std::vector<double> &sn, const std::vector<double> &g);
// y = a*x + b*y (y is not read when b == 0)
hipError_t launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t st);
// y = x + lam*d
hipError_t launch_xpld(int64_t n, const double *x, double lam, const double *d, double *y,
                       hipStream_t st);
// y = x / s[0] (s on device)
hipError_t launch_scale_div(int64_t n, const double *x, const double *s, double *y,
                            hipStream_t st);
// y += sum_j c[j] Z_j with Z of type Tz (c on device)
template <typename Tz>
hipError_t launch_combine(const Tz *Z, int64_t ld, int k, const double *c, double *y, int64_t n,
                          hipStream_t st);
template <typename Ta, typename Tb>
hipError_t launch_cast(const Ta *a, Tb *b, int64_t n, hipStream_t st);
hipError_t launch_compliance(const Geo &g, const double *x, const double *s,
                             const uint8_t *nmask, double *dfdx, double *partial,
                             hipStream_t st);

// ---- errors ----------------------------------------------------------------
void set_error(const std::string &msg);
int hip_fail(hipError_t e, const char *what);

struct SolverWs;
struct Mg;
struct BatchEngine;

// One FGMRES solve A x = b handed to the batch engine (lockstep Krylov
// iterations over all solves in flight; fe_batch.cpp).  The caller fills the
// inputs, keeps every buffer alive and untouched until batch_fgmres returns.
struct BJob {
    fe_problem *p = nullptr;
    Mg *mg = nullptr;                 // multigrid hierarchy, set up for this Newton step
    bool mixed = false;               // FP32 V-cycle and J z (GMRES-IR), FP64 otherwise
    bool pc32 = false;                // (not mixed) FP32 V-cycle, z_j kept in FP32, FP64 J z
    const double *b = nullptr;        // right-hand side
    double *x = nullptr;              // solution (set to 0 first)
    const double *xlin = nullptr;     // linearisation state
    const float *x32 = nullptr;       // its FP32 copy (mixed)
    const double *gamma = nullptr, *s = nullptr;
    double *V = nullptr, *Z = nullptr, *tmp = nullptr, *partial = nullptr;
    float *Z32 = nullptr;
    int64_t n = 0;
    int m = 0, max_its = 0, n_refine = 0;
    double rtol = 0.0;
    hipEvent_t ready = nullptr;       // recorded on the caller's stream at submission
    // results
    int rc = 0, its = 0;
    bool converged = false, done = false;
    double res_true = 0.0;
    std::string error;
    std::condition_variable cv;       // the submitting worker waits here for done
};
int batch_engine_create(int device, BatchEngine **out);
void batch_engine_destroy(BatchEngine *E);
// Solve job on the engine; blocks until it is finished (its work on the device
// complete).  st: the caller's stream, on which the inputs were produced.
int batch_fgmres(BatchEngine *E, BJob *job, hipStream_t st);
void batch_engine_stats(const BatchEngine *E, uint64_t *steps, uint64_t *launches);

// Device / host memory source of a problem: hipMalloc by default, or a
// sub-allocator over a pre-allocated HBM arena (the solve server).
struct Allocator {
    virtual ~Allocator() = default;
    virtual hipError_t dev_alloc(void **p, size_t n) = 0;
    virtual void dev_free(void *p) = 0;
    virtual hipError_t host_alloc(void **p, size_t n) = 0;  // host staging memory
    virtual void host_free(void *p) = 0;
};
Allocator *default_allocator();

enum MaskKind { MASK_GIVEN = 0, MASK_WALLS_PIN = 1 };
// Internal constructor: mask from a device array (MASK_GIVEN, may be NULL) or
// generated on the device (walls u,v,w,T plus the pressure of node 0);
// allocations through alloc, set-up work ordered on stream.
int problem_create_ex(const fe_grid *grid, const fe_phys *phys, const uint8_t *dof_mask,
                      MaskKind kind, Allocator *alloc, hipStream_t stream, fe_problem **out);
hipError_t launch_wall_mask(int nx, int ny, int nz, uint8_t *nmask, uint8_t *dof_mask,
                            hipStream_t st);

}  // namespace fe

struct fe_problem {
    fe_grid grid;
    fe_phys phys;
    fe::Geo geo;
    int device;
    int64_t nn, ne, ndof;
    uint8_t *nmask = nullptr;     // per node: bit f = DOF f prescribed
    uint8_t *dof_mask = nullptr;  // per DOF copy of the caller's mask
    double *slots = nullptr;      // tile-face partial sums (5 values / node box entry)
    double *slots25 = nullptr;    // block-diagonal partial sums (25 values)
    double *partial = nullptr;    // reduction partials, PARTIAL_COLS * RED_BLOCKS
    double *scal = nullptr;       // device scalars
    fe::SolverWs *ws = nullptr;    // Newton/FGMRES workspace (allocated on first solve)
    fe::BatchEngine *batch = nullptr; // if set, Newton's multigrid FGMRES solves run on it
    fe::Allocator *alloc = nullptr; // memory source of this problem's buffers
    // Element-pass timer of fe_jvp (instrumentation, off by default): start/stop
    // event pairs, timer_n of them recorded since the last read.
    bool timer_on = false;
    std::vector<hipEvent_t> timer_ev;
    size_t timer_n = 0;
};

namespace fe {
template <typename T>
inline hipError_t dalloc(fe_problem *p, T **ptr, size_t bytes)
{
    return p->alloc->dev_alloc(reinterpret_cast<void **>(ptr), bytes);
}
inline void dfree(fe_problem *p, void *ptr)
{
    if (ptr) p->alloc->dev_free(ptr);
}
template <typename T>
inline hipError_t halloc(fe_problem *p, T **ptr, size_t bytes)
{
    return p->alloc->host_alloc(reinterpret_cast<void **>(ptr), bytes);
}
inline void hfree(fe_problem *p, void *ptr)
{
    if (ptr) p->alloc->host_free(ptr);
}
}  // namespace fe

#define FE_CHECK_HIP(call)                                        \
    do {                                                          \
        hipError_t _e = (call);                                   \
        if (_e != hipSuccess) return fe::hip_fail(_e, #call);     \
    } while (0)
