// Lockstep Krylov engine of the batched solve server.
//
// Every Newton step of a served request needs one linear solve J d = -R
// (Sec. "Solving the non-linear system": flexible GMRES, preconditioned by a
// geometric multigrid V-cycle).  The requests' worker threads hand these solves
// to one engine thread, which advances all of them together: each engine step
// performs one action per solve -- start (x = 0, |b|, c_0 = b / |b|), one
// FGMRES iteration (V-cycle, J z, the dot and update passes of classical
// Gram-Schmidt with the second projection delayed by a step), the candidate's
// dot pass alone that finishes the last Hessenberg column of a cycle, or the
// end of a cycle (x += Z y, then in mixed mode or when the estimate has not
// converged the true residual b - J x and its norm) -- and
// every kernel of the step runs as ONE batched launch over the table of all
// solves that need it, whatever their grid sizes.  A step ends with one copy
// of the solves' small results (Hessenberg column, norms) to the host, where
// each solve's Givens rotations and convergence tests run exactly as in the
// one-problem FGMRES.  Set-up (block diagonals, coarse operators) and the
// Newton line search stay with the worker threads, on their own streams.
//
// A solve's arithmetic does not depend on the other solves of a step: the
// element and multigrid kernels are the one-problem kernels' bodies, and the
// reductions chunk each vector by its own length.  Its result is therefore the
// same alone and in any mix.  It follows the one-problem FGMRES step for step;
// only the reductions are chunked differently, so the two agree to rounding,
// not bitwise.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "fe_batch.h"
#include "fe_internal.h"
#include "fe_mg.h"

namespace fe {

namespace {

constexpr int MAX_SLOTS = 512;   // solves in flight at once
constexpr int RS = 136;          // result doubles per slot: Gram-Schmidt products (2j + 9), or
constexpr int R_BETA = 130, R_NRM2 = 131;  // |b| and |b|^2 of a start / cycle end
constexpr int MAXD = 64;         // depth bound of the V-cycle phase keys

// launch kinds
enum Kind {
    K_FILL, K_CAST, K_AXPBY, K_SCALE, K_COMB64, K_COMB32, K_DOTS, K_REDUCE, K_DGSD, K_DGSU, K_SCNORM,
    K_EJV_DD, K_CJV_DD, K_EJV_FD, K_CJV_FD, K_EJV_FF, K_CJV_FF,
    K_ESM_D, K_CSM_D, K_ESM_F, K_CSM_F,
    K_ST_D, K_ST_F, K_SM0_D, K_SM0_F, K_SM1_D, K_SM1_F,
    K_RS_D, K_RS_F, K_RSS_D, K_RSS_F, K_PR_D, K_PR_F,
    K_CP_D, K_CP_F, K_CS_D, K_CS_F,
    K_SS_D, K_SS_F, K_SM0C, K_CPY_D, K_CPY_F, K_WIDEN,
    K_COUNT
};
using LaunchFn = hipError_t (*)(const BLaunch &, hipStream_t);
const LaunchFn kLaunch[K_COUNT] = {
    blaunch_fill, blaunch_cast, blaunch_axpby, blaunch_scale, blaunch_comb<double>,
    blaunch_comb<float>, blaunch_dots, blaunch_reduce, blaunch_dgs_dots, blaunch_dgs_update,
    blaunch_scale_norm,
    blaunch_elem_jv<double, double>, blaunch_combine_jv<double, double>,
    blaunch_elem_jv<float, double>, blaunch_combine_jv<float, double>,
    blaunch_elem_jv<float, float>, blaunch_combine_jv<float, float>,
    blaunch_elem_smooth_pass<double>, blaunch_combine_smooth<double>,
    blaunch_elem_smooth_pass<float>, blaunch_combine_smooth<float>,
    blaunch_stencil<double>, blaunch_stencil<float>,
    blaunch_smooth<double, false>, blaunch_smooth<float, false>,
    blaunch_smooth<double, true>, blaunch_smooth<float, true>,
    blaunch_restrict<double>, blaunch_restrict<float>,
    blaunch_restrict_smooth<double>, blaunch_restrict_smooth<float>,
    blaunch_prolong<double>, blaunch_prolong<float>,
    blaunch_coarse_part<double>, blaunch_coarse_part<float>,
    blaunch_coarse_sum<double>, blaunch_coarse_sum<float>,
    blaunch_stencil_smooth<double>, blaunch_stencil_smooth<float>, blaunch_smooth0_cast,
    blaunch_copy<double>, blaunch_copy<float>, blaunch_widen,
};

// Kind of a templated kernel for T = double / float.
template <typename T>
constexpr int kd(int kdouble, int kfloat)
{
    return sizeof(T) == 8 ? kdouble : kfloat;
}

// Phase key: segment (0 start / cycle end, 1 V-cycle down, 2 V-cycle up,
// 3 operator and Gram-Schmidt), level order within the segment, stage.
constexpr uint64_t key(int seg, int lvl, int stage)
{
    return ((uint64_t)seg << 40) | ((uint64_t)lvl << 20) | (uint64_t)stage;
}

// The step's launches: ops are collected per solve in dependency order, then
// grouped by (key, kind) -- one batched launch per group, in key order.
struct Planner {
    struct Op {
        uint64_t key;
        int kind;
        int nblk;
        size_t arg_off, arg_size;
        int seq;
    };
    std::vector<Op> ops;
    std::vector<char> args;

    void clear()
    {
        ops.clear();
        args.clear();
    }
    template <class A>
    void add(uint64_t k, int kind, const A &a, int nblk)
    {
        if (nblk <= 0) return;
        const size_t off = args.size();
        args.resize(off + sizeof(A));
        std::memcpy(args.data() + off, &a, sizeof(A));
        ops.push_back(Op{k, kind, nblk, off, sizeof(A), (int)ops.size()});
    }
};

enum JState { J_INIT, J_ITER, J_FINAL, J_CEND };

struct Solve {
    BJob *job = nullptr;
    int slot = -1;
    JState state = J_INIT;
    int m = 0, j = 0, kk = 0, refine_left = 0;
    std::vector<double> H, cs, sn, g, y;
    std::vector<double> Hp;  // provisional column j - 1 (first-projection coefficients)
    double om = 0, c2 = 0;   // scale and squared norm of the candidate c_j
    bool col_final = false;  // column j - 1 was finished before step j (J_FINAL)
    double beta0 = 0, target = 0, res = 0;
    bool breakdown = false, est_conv = false, need_true = false, waited = false;
};

template <typename T>
T *vec_of(MgLevel &L, int which);
template <>
double *vec_of<double>(MgLevel &L, int which)
{
    return which == 0 ? L.b : which == 1 ? L.xs : L.t;
}
template <>
float *vec_of<float>(MgLevel &L, int which)
{
    return which == 0 ? L.b32 : which == 1 ? L.xs32 : L.t32;
}
template <typename T>
const T *state_of(const MgLevel &L)
{
    if constexpr (sizeof(T) == 8)
        return L.x;
    else
        return L.x32;
}
template <typename T>
const T *blocks_of(const MgLevel &L)
{
    if constexpr (sizeof(T) == 8)
        return L.D;
    else
        return L.D32;
}
template <typename T>
const T *stencil_of(const MgLevel &L)
{
    if constexpr (sizeof(T) == 8)
        return L.S;
    else
        return L.S32;
}

// t = A x on level L (assembled stencil, or element pass + shared-node pass)
template <typename T>
void emit_op(Planner &P, uint64_t k, MgLevel &L, const T *x, T *t)
{
    if (L.assembled) {
        P.add(k, kd<T>(K_ST_D, K_ST_F),
              BStencil<T>{L.grid.nx, L.grid.ny, L.grid.nz, stencil_of<T>(L), x, t},
              bstencil_blocks(L.nn));
        return;
    }
    const BElem<T, T> a{L.geo, state_of<T>(L), x, L.gamma, L.s, L.nmask, t, (T *)L.slots};
    P.add(k, kd<T>(K_EJV_DD, K_EJV_FF), a, belem_blocks(L.geo));
    P.add(k + 1, kd<T>(K_CJV_DD, K_CJV_FF), a, bnode_blocks(L.geo));
}

template <typename T>
T *alt_of(MgLevel &L)
{
    if constexpr (sizeof(T) == 8)
        return L.xa;
    else
        return L.xa32;
}

// x += omega D^{-1} (b - A x) on level L: the element pass and the fused
// shared-node/smoothing pass in place on matrix-free levels; one kernel on
// assembled ones, writing the other of the level's two iterate buffers (x, the
// level's own, and its second buffer); cur tracks where the iterate is.
template <typename T>
void emit_sweep(Planner &P, uint64_t k, MgLevel &L, const T *D, const T *b, T *x, T *&cur, T *t, T om)
{
    if (L.assembled) {
        T *nxt = cur == x ? alt_of<T>(L) : x;
        P.add(k, kd<T>(K_SS_D, K_SS_F),
              BStencilSmooth<T>{L.grid.nx, L.grid.ny, L.grid.nz, stencil_of<T>(L), D, b, cur, nxt, om},
              bstencil_smooth_blocks(L.nn));
        cur = nxt;
        return;
    }
    const BElemSmooth<T> a{L.geo, state_of<T>(L), cur, L.gamma, L.s, L.nmask, t, (T *)L.slots, D, b,
                           om};
    P.add(k, kd<T>(K_ESM_D, K_ESM_F), a, belem_blocks(L.geo));
    P.add(k + 1, kd<T>(K_CSM_D, K_CSM_F), a, bnode_blocks(L.geo));
}

// z = M v, one V-cycle in the precision of T (the same sequence as the
// one-problem V-cycle: first sweep from zero, nu1 - 1 more, residual,
// restriction -- fused with the next level's first sweep except above the
// directly solved level --, coarse solve, prolongation, nu2 sweeps)
template <typename T>
void emit_vcycle(Planner &P, Mg *mg, const double *v, T *z)
{
    const int nl = (int)mg->lev.size();
    const T om = (T)mg->omega;
    std::vector<const T *> bl(nl);
    std::vector<T *> xl(nl), cur(nl);
    bool first_done = false;
    if constexpr (sizeof(T) == 4) {
        // the first sweep from zero reads the FP64 Krylov vector and keeps its cast
        MgLevel &L0 = mg->lev[0];
        P.add(key(1, 0, 1), K_SM0C, BSmooth0Cast{L0.D32, v, L0.b32, z, L0.nn, om},
              bsmooth_blocks(L0.nn));
        bl[0] = L0.b32;
        first_done = true;
    } else {
        bl[0] = v;
    }
    xl[0] = z;
    for (int l = 0; l + 1 < nl; ++l) {
        MgLevel &L = mg->lev[l], &C = mg->lev[l + 1];
        const T *D = blocks_of<T>(L);
        T *t = vec_of<T>(L, 2);
        cur[l] = xl[l];
        if (!first_done)
            P.add(key(1, l, 1), kd<T>(K_SM0_D, K_SM0_F), BSmooth<T>{D, bl[l], nullptr, xl[l], L.nn, om},
                  bsmooth_blocks(L.nn));
        for (int it = 1; it < mg->nu1; ++it)
            emit_sweep<T>(P, key(1, l, 2 * it), L, D, bl[l], xl[l], cur[l], t, om);
        emit_op<T>(P, key(1, l, 40), L, cur[l], t);
        T *bc = vec_of<T>(C, 0), *xc = vec_of<T>(C, 1);
        bl[l + 1] = bc;
        xl[l + 1] = xc;
        const bool fuse = l + 2 < nl;
        BRestrict<T> r{C.grid.nx, C.grid.ny, C.grid.nz, L.grid.nx, L.grid.ny, L.grid.nz,
                       bl[l],     t,         C.nmask,   bc,        nullptr,   nullptr,   om};
        if (fuse) {
            r.Dc = blocks_of<T>(C);
            r.xc = xc;
            P.add(key(1, l, 42), kd<T>(K_RSS_D, K_RSS_F), r, brestrict_smooth_blocks(C.nn));
        } else {
            P.add(key(1, l, 42), kd<T>(K_RS_D, K_RS_F), r, brestrict_blocks(C.nn));
            const int nf = (int)mg->nf;
            const BCoarse<T> c{(int)mg->nc, nf, (nf + 63) / 64, mg->Xinv, mg->dmap,
                               mg->dmap + mg->nc, bc, xc, mg->cpart};
            P.add(key(1, l, 43), kd<T>(K_CP_D, K_CP_F), c, bcoarse_part_blocks(nf));
            P.add(key(1, l, 44), kd<T>(K_CS_D, K_CS_F), c, bcoarse_sum_blocks((int)mg->nc));
        }
        first_done = fuse;
    }
    for (int l = nl - 2; l >= 0; --l) {
        MgLevel &L = mg->lev[l], &C = mg->lev[l + 1];
        const T *D = blocks_of<T>(L);
        T *t = vec_of<T>(L, 2);
        P.add(key(2, MAXD - l, 0), kd<T>(K_PR_D, K_PR_F),
              BProlong<T>{L.grid.nx, L.grid.ny, L.grid.nz, C.grid.nx, C.grid.ny, xl[l + 1], L.nmask,
                          cur[l]},
              bprolong_blocks(L.nn));
        for (int it = 0; it < mg->nu2; ++it)
            emit_sweep<T>(P, key(2, MAXD - l, 1 + 2 * it), L, D, bl[l], xl[l], cur[l], t, om);
        if (cur[l] != xl[l])
            P.add(key(2, MAXD - l, 39), kd<T>(K_CPY_D, K_CPY_F), BCopy<T>{cur[l], xl[l], L.ndof},
                  belt_blocks(L.ndof));
    }
}

// |w| into the slot (norm2, beta) and v = w / |w|
void emit_norm_scale(Planner &P, int stage, const BJob &J, double *res, const double *w, double *v)
{
    int nch, ept;
    bred_chunks(J.n, &nch, &ept);
    P.add(key(0, 0, stage), K_DOTS, BDots{w, nullptr, J.n, 0, 1, J.n, nch, ept, 1, J.partial}, nch);
    P.add(key(0, 0, stage + 1), K_SCNORM,
          BScaleNorm{J.partial, nch, J.n, w, v, res + R_NRM2, res + R_BETA}, belt_blocks(J.n));
}

// Delayed Gram-Schmidt with J basis vectors: the dot pass (with the new
// Krylov vector when w, else the candidate's products alone) reduced into the
// slot, and with w the update pass and the next candidate's |c|^2 (slot 2J + 8).
void emit_dgs(Planner &P, const BJob &J, double *res, int nb, bool w)
{
    int nch, ept;
    bred_chunks(J.n, &nch, &ept);
    const int ngrp = std::max(1, (nb + BDOT_GROUP - 1) / BDOT_GROUP);
    P.add(key(3, 0, 10), K_DGSD, BDgsDots{J.V, J.n, nb, w ? 1 : 0, J.n, nch, ept, ngrp, J.partial},
          nch * ngrp);
    const int ncol = w ? 2 * nb + 3 : nb + 1;
    P.add(key(3, 0, 11), K_REDUCE, BReduce{J.partial, ncol, nch, res, nullptr}, ncol);
    if (!w) return;
    P.add(key(3, 0, 12), K_DGSU, BDgsUpdate{J.V, J.n, nb, J.n, nch, ept, res, J.partial}, nch);
    P.add(key(3, 0, 13), K_REDUCE, BReduce{J.partial, 1, nch, res + 2 * nb + 8, nullptr}, 1);
}

}  // namespace

struct BatchEngine {
    int device = 0;
    hipStream_t st = nullptr;
    double *dres = nullptr, *hres = nullptr;
    char *dstage = nullptr, *hstage = nullptr;
    size_t stage_cap = 0;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;       // work arrived / stop
    std::vector<BJob *> incoming;
    bool stop = false;
    std::vector<Solve> active;
    std::vector<int> free_slots;
    Planner P;
    std::atomic<uint64_t> steps{0}, launches{0};  // read by other threads (batch_engine_stats)

    int ensure_stage(size_t bytes)
    {
        if (bytes <= stage_cap) return FE_OK;
        size_t cap = std::max<size_t>(bytes * 2, (size_t)4 << 20);
        if (dstage) (void)hipFree(dstage);
        if (hstage) (void)hipHostFree(hstage);
        dstage = nullptr;
        hstage = nullptr;
        stage_cap = 0;
        hipError_t e = hipMalloc(&dstage, cap);
        if (e == hipSuccess) e = hipHostMalloc(&hstage, cap);
        if (e != hipSuccess) return hip_fail(e, "batch engine: staging buffers");
        stage_cap = cap;
        return FE_OK;
    }

    double *slot_res(int slot) { return dres + (size_t)slot * RS; }
    const double *slot_hres(int slot) const { return hres + (size_t)slot * RS; }

    void plan(Solve &S);
    int execute();
    void update(Solve &S, bool *finished);
    void run();
};

void BatchEngine::plan(Solve &S)
{
    const BJob &J = *S.job;
    double *res = slot_res(S.slot);
    const int64_t n = J.n;
    switch (S.state) {
    case J_INIT:
        P.add(key(0, 0, 0), K_FILL, BFill{J.x, n}, belt_blocks(n));
        emit_norm_scale(P, 8, J, res, J.b, J.V);
        break;
    case J_CEND: {
        if (J.mixed || J.pc32) {  // z_j stored in FP32
            BComb<float> c{J.Z32, n, S.kk, n, J.x, {}};
            std::copy(S.y.begin(), S.y.begin() + S.kk, c.y);
            P.add(key(0, 0, 4), K_COMB32, c, belt_blocks(n));
        } else {
            BComb<double> c{J.Z, n, S.kk, n, J.x, {}};
            std::copy(S.y.begin(), S.y.begin() + S.kk, c.y);
            P.add(key(0, 0, 4), K_COMB64, c, belt_blocks(n));
        }
        if (S.need_true && !(J.its >= J.max_its && !S.est_conv)) {
            const fe_problem *p = J.p;
            const BElem<double, double> a{p->geo, J.xlin, J.x, J.gamma, J.s, p->nmask, J.tmp, p->slots};
            P.add(key(0, 0, 5), K_EJV_DD, a, belem_blocks(p->geo));
            P.add(key(0, 0, 6), K_CJV_DD, a, bnode_blocks(p->geo));
            P.add(key(0, 0, 7), K_AXPBY, BAxpby{n, 1.0, J.b, -1.0, J.tmp}, belt_blocks(n));
            emit_norm_scale(P, 8, J, res, J.tmp, J.V);
        }
        break;
    }
    case J_ITER: {
        const fe_problem *p = J.p;
        double *vj = J.V + (int64_t)S.j * n, *vn = J.V + (int64_t)(S.j + 1) * n;
        if (J.mixed) {
            float *zj = J.Z32 + (int64_t)S.j * n;
            emit_vcycle<float>(P, J.mg, vj, zj);
            const BElem<float, double> a{p->geo, J.x32, zj, J.gamma, J.s, p->nmask, vn, p->slots};
            P.add(key(3, 0, 0), K_EJV_FD, a, belem_blocks(p->geo));
            P.add(key(3, 0, 1), K_CJV_FD, a, bnode_blocks(p->geo));
        } else if (J.pc32) {
            // FP32 V-cycle into the FP32 column, widened into the (otherwise
            // unused) FP64 column after the cycle's last phase, FP64 J z
            float *zj = J.Z32 + (int64_t)S.j * n;
            double *zw = J.Z + (int64_t)S.j * n;
            emit_vcycle<float>(P, J.mg, vj, zj);
            P.add(key(2, MAXD, 50), K_WIDEN, BWiden{zj, zw, n}, belt_blocks(n));
            const BElem<double, double> a{p->geo, J.xlin, zw, J.gamma, J.s, p->nmask, vn, p->slots};
            P.add(key(3, 0, 0), K_EJV_DD, a, belem_blocks(p->geo));
            P.add(key(3, 0, 1), K_CJV_DD, a, bnode_blocks(p->geo));
        } else {
            double *zj = J.Z + (int64_t)S.j * n;
            emit_vcycle<double>(P, J.mg, vj, zj);
            const BElem<double, double> a{p->geo, J.xlin, zj, J.gamma, J.s, p->nmask, vn, p->slots};
            P.add(key(3, 0, 0), K_EJV_DD, a, belem_blocks(p->geo));
            P.add(key(3, 0, 1), K_CJV_DD, a, bnode_blocks(p->geo));
        }
        emit_dgs(P, J, res, S.j, true);
        break;
    }
    case J_FINAL:
        emit_dgs(P, J, res, S.j, false);
        break;
    }
}

// Group the planned ops into batched launches, upload their tables in one
// copy, launch, and copy the slots' results back (synchronises the stream).
int BatchEngine::execute()
{
    std::vector<Planner::Op> &ops = P.ops;
    std::sort(ops.begin(), ops.end(), [](const Planner::Op &a, const Planner::Op &b) {
        if (a.key != b.key) return a.key < b.key;
        if (a.kind != b.kind) return a.kind < b.kind;
        return a.seq < b.seq;
    });
    struct Grp {
        int kind, n, blocks;
        size_t tab, off;
    };
    std::vector<Grp> grps;
    auto align = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t need = 0;
    for (size_t i = 0; i < ops.size();) {
        size_t e = i;
        while (e < ops.size() && ops[e].key == ops[i].key && ops[e].kind == ops[i].kind) ++e;
        const size_t cnt = e - i;
        need = align(need) + cnt * ops[i].arg_size;
        need = align(need) + (cnt + 1) * sizeof(int);
        i = e;
    }
    int rc = ensure_stage(need + 256);
    if (rc) return rc;
    size_t pos = 0;
    for (size_t i = 0; i < ops.size();) {
        size_t e = i;
        while (e < ops.size() && ops[e].key == ops[i].key && ops[e].kind == ops[i].kind) ++e;
        Grp gr{ops[i].kind, (int)(e - i), 0, 0, 0};
        pos = align(pos);
        gr.tab = pos;
        for (size_t q = i; q < e; ++q) {
            std::memcpy(hstage + pos, P.args.data() + ops[q].arg_off, ops[q].arg_size);
            pos += ops[q].arg_size;
        }
        pos = align(pos);
        gr.off = pos;
        int *off = reinterpret_cast<int *>(hstage + pos);
        off[0] = 0;
        for (size_t q = i; q < e; ++q) off[q - i + 1] = off[q - i] + ops[q].nblk;
        gr.blocks = off[e - i];
        pos += (e - i + 1) * sizeof(int);
        grps.push_back(gr);
        i = e;
    }
    if (pos > 0) FE_CHECK_HIP(hipMemcpyAsync(dstage, hstage, pos, hipMemcpyHostToDevice, st));
    for (const Grp &gr : grps) {
        BLaunch L;
        L.tab = dstage + gr.tab;
        L.off = reinterpret_cast<const int *>(dstage + gr.off);
        L.n = gr.n;
        L.blocks = gr.blocks;
        FE_CHECK_HIP(kLaunch[gr.kind](L, st));
    }
    launches += grps.size();
    int top = 0;
    for (const Solve &S : active) top = std::max(top, S.slot + 1);
    if (top > 0)
        FE_CHECK_HIP(hipMemcpyAsync(hres, dres, sizeof(double) * RS * top, hipMemcpyDeviceToHost, st));
    FE_CHECK_HIP(hipStreamSynchronize(st));
    return FE_OK;
}

// Host side of a step for one solve: the same decisions as the one-problem FGMRES.
void BatchEngine::update(Solve &S, bool *finished)
{
    BJob &J = *S.job;
    const double *hh = slot_hres(S.slot);
    const int m = S.m;
    auto finish = [&](int rc) {
        J.rc = rc;
        *finished = true;
    };
    // the cycle ends with kk final columns: y = H^{-1} g, then the cycle-end step
    auto end_cycle = [&](int kk) {
        for (int i = kk - 1; i >= 0; --i) {
            double s = S.g[i];
            for (int c = i + 1; c < kk; ++c) s -= S.H[(size_t)i * m + c] * S.y[c];
            S.y[i] = s / S.H[(size_t)i * m + i];
        }
        S.kk = kk;
        S.est_conv = S.res <= S.target;
        S.need_true = J.mixed || !S.est_conv;
        S.state = J_CEND;
    };
    // before step j: finish column j - 1 from the candidate's dot products
    // alone (J_FINAL) when the step would not be used, else take the step
    auto next_step = [&]() {
        const int j = S.j;
        if (j == 0) {
            if (J.its >= J.max_its)
                end_cycle(0);
            else
                S.state = J_ITER;
            return;
        }
        bool fin = j == m || J.its >= J.max_its;
        if (!fin) {
            S.Hp[j] = S.om * std::sqrt(std::max(S.c2, 0.0));
            fin = givens_estimate(S.Hp, j - 1, S.cs, S.sn, S.g) <= S.target;
        }
        S.state = fin ? J_FINAL : J_ITER;
    };
    auto start_cycle = [&](double beta) {
        std::fill(S.g.begin(), S.g.end(), 0.0);
        S.j = 0;
        S.om = beta;
        S.c2 = 1.0;
        S.res = beta;
        S.breakdown = false;
        S.col_final = false;
        next_step();
    };
    // column j - 1 from its provisional entries, the candidate's s and sigma
    auto finish_column = [&](int j, const double *s, double sig) {
        for (int i = 0; i < j; ++i) S.H[(size_t)i * m + (j - 1)] = S.Hp[i] + S.om * s[i];
        S.H[(size_t)j * m + (j - 1)] = S.om * sig;
        S.res = givens_column(S.H, m, j - 1, S.cs, S.sn, S.g);
        if (!(S.om * sig > 1e-300 * S.beta0)) S.breakdown = true;
    };
    switch (S.state) {
    case J_INIT: {
        const double beta0 = hh[R_BETA];
        J.its = 0;
        J.converged = false;
        if (!std::isfinite(beta0)) {
            J.error = "non-finite right-hand side in FGMRES";
            finish(FE_ENAN);
            return;
        }
        if (beta0 == 0.0) {
            J.converged = true;
            finish(FE_OK);
            return;
        }
        S.beta0 = beta0;
        S.target = J.rtol * beta0;
        S.refine_left = J.n_refine;
        start_cycle(beta0);
        return;
    }
    case J_ITER: {
        const int j = S.j;
        const double sig = hh[2 * j + 3], hj = hh[2 * j + 4], omn = hh[2 * j + 5];
        const double cn2 = hh[2 * j + 8];
        J.its++;
        if (!std::isfinite(sig) || !std::isfinite(hj) || !std::isfinite(omn) || !std::isfinite(cn2)) {
            J.error = "non-finite Krylov norm";
            finish(FE_ENAN);
            return;
        }
        if (j == 0) {
            S.g[0] = S.om * sig;
            if (!(sig > 0.0)) S.breakdown = true;
        } else if (!S.col_final) {
            finish_column(j, hh, sig);
        }
        S.col_final = false;
        if (S.breakdown || (j >= 1 && S.res <= S.target)) {
            end_cycle(j);
            return;
        }
        for (int i = 0; i < j; ++i) S.Hp[i] = hh[j + 1 + i];
        S.Hp[j] = hj;
        S.om = omn;
        S.c2 = cn2;
        S.j = j + 1;
        next_step();
        return;
    }
    case J_FINAL: {
        const int j = S.j;
        double ss = 0.0;
        for (int i = 0; i < j; ++i) ss += hh[i] * hh[i];
        const double s2 = hh[j] - ss;
        if (!std::isfinite(s2)) {
            J.error = "non-finite Krylov norm";
            finish(FE_ENAN);
            return;
        }
        finish_column(j, hh, s2 > 0.0 ? std::sqrt(s2) : 0.0);
        if (S.res <= S.target || J.its >= J.max_its || j == m || S.breakdown) {
            end_cycle(j);
        } else {
            // the estimate was optimistic: take step j, whose dot pass must not
            // finish column j - 1 (and rotate g) a second time
            S.col_final = true;
            S.state = J_ITER;
        }
        return;
    }
    case J_CEND: {
        if (J.its >= J.max_its && !S.est_conv) {
            finish(FE_OK);
            return;
        }
        if (!S.need_true) {
            J.converged = true;
            J.res_true = S.res;
            finish(FE_OK);
            return;
        }
        const double beta = hh[R_BETA];
        J.res_true = beta;
        if (beta <= S.target) {
            J.converged = true;
            finish(FE_OK);
            return;
        }
        if (S.est_conv && S.refine_left-- <= 0) {
            finish(FE_OK);
            return;
        }
        if (J.its >= J.max_its || S.breakdown) {
            finish(FE_OK);
            return;
        }
        start_cycle(beta);  // c_0 = r / |r| was formed on the device in this step
        return;
    }
    }
}

void BatchEngine::run()
{
    (void)hipSetDevice(device);
    while (true) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return stop || !incoming.empty() || !active.empty(); });
            if (stop && incoming.empty() && active.empty()) break;
            // solves beyond the free result slots wait for the next step
            size_t taken = 0;
            for (BJob *jb : incoming) {
                if (free_slots.empty()) break;
                ++taken;
                Solve S;
                S.job = jb;
                S.slot = free_slots.back();
                free_slots.pop_back();
                S.m = jb->m;
                S.H.assign((size_t)(S.m + 1) * S.m, 0.0);
                S.cs.assign(S.m, 0.0);
                S.sn.assign(S.m, 0.0);
                S.g.assign(S.m + 1, 0.0);
                S.y.assign(S.m, 0.0);
                S.Hp.assign(S.m + 2, 0.0);
                active.push_back(std::move(S));
            }
            incoming.erase(incoming.begin(), incoming.begin() + taken);
        }
        // the solves' inputs were produced on their workers' streams
        for (Solve &S : active)
            if (!S.waited) {
                (void)hipStreamWaitEvent(st, S.job->ready, 0);
                S.waited = true;
            }
        P.clear();
        for (Solve &S : active) plan(S);
        const int rc = execute();
        ++steps;
        std::vector<Solve> keep;
        keep.reserve(active.size());
        std::vector<BJob *> done;
        for (Solve &S : active) {
            bool fin = false;
            if (rc) {
                S.job->rc = rc;
                S.job->error = fe_last_error();
                fin = true;
            } else {
                update(S, &fin);
            }
            if (fin)
                done.push_back(S.job);
            else
                keep.push_back(std::move(S));
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            for (Solve &S : active) {
                bool gone = true;
                for (const Solve &K : keep)
                    if (K.slot == S.slot) gone = false;
                if (gone) free_slots.push_back(S.slot);
            }
            active.swap(keep);
            // only the finished solves' workers are woken; notified under the
            // lock, since a woken worker returns and its job object ends
            for (BJob *jb : done) {
                jb->done = true;
                jb->cv.notify_one();
            }
        }
    }
}

int batch_engine_create(int device, BatchEngine **out)
{
    *out = nullptr;
    auto *E = new (std::nothrow) BatchEngine();
    if (!E) return FE_ENOMEM;
    E->device = device;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&E->st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&E->dres, sizeof(double) * RS * MAX_SLOTS);
    if (e == hipSuccess) e = hipHostMalloc(&E->hres, sizeof(double) * RS * MAX_SLOTS);
    if (e != hipSuccess) {
        batch_engine_destroy(E);
        return hip_fail(e, "batch engine: creation");
    }
    int rc = E->ensure_stage((size_t)4 << 20);
    if (rc) {
        batch_engine_destroy(E);
        return rc;
    }
    for (int s = MAX_SLOTS - 1; s >= 0; --s) E->free_slots.push_back(s);
    E->th = std::thread([E] { E->run(); });
    *out = E;
    return FE_OK;
}

void batch_engine_destroy(BatchEngine *E)
{
    if (!E) return;
    if (E->th.joinable()) {
        {
            std::lock_guard<std::mutex> lk(E->mu);
            E->stop = true;
        }
        E->cv.notify_all();
        E->th.join();
    }
    if (E->dstage) (void)hipFree(E->dstage);
    if (E->hstage) (void)hipHostFree(E->hstage);
    if (E->dres) (void)hipFree(E->dres);
    if (E->hres) (void)hipHostFree(E->hres);
    if (E->st) (void)hipStreamDestroy(E->st);
    delete E;
}

int batch_fgmres(BatchEngine *E, BJob *job, hipStream_t st)
{
    if (job->m < 1 || job->m > BCOMB_MAX) {
        set_error("batched FGMRES: restart length must be 1..64");
        return FE_EINVAL;
    }
    job->done = false;
    job->rc = FE_OK;
    job->its = 0;
    job->converged = false;
    job->res_true = 0.0;
    FE_CHECK_HIP(hipEventRecord(job->ready, st));
    {
        std::unique_lock<std::mutex> lk(E->mu);
        E->incoming.push_back(job);
        E->cv.notify_all();
        job->cv.wait(lk, [&] { return job->done; });
    }
    if (job->rc != FE_OK && !job->error.empty()) set_error(job->error);
    return job->rc;
}

void batch_engine_stats(const BatchEngine *E, uint64_t *steps, uint64_t *launches)
{
    if (steps) *steps = E ? E->steps.load() : 0;
    if (launches) *launches = E ? E->launches.load() : 0;
}

}  // namespace fe

struct fe_batch {
    fe_prec prec = FE_FP64;
    int n = 0;
    void *dtab = nullptr;  // table, then element-pass offsets, then shared-node offsets
    fe::BLaunch elem, comb;
};

namespace {

template <typename T>
int jvp_batch_build(fe_batch *B, int n, fe_problem *const *probs, const void *const *x,
                    const double *const *gamma, const double *const *s, const void *const *v,
                    void *const *jv)
{
    using namespace fe;
    std::vector<BElem<T, T>> tab(n);
    std::vector<int> oe(n + 1, 0), oc(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        fe_problem *p = probs[i];
        tab[i] = BElem<T, T>{p->geo, (const T *)x[i], (const T *)v[i], gamma[i], s[i], p->nmask,
                             (T *)jv[i], (T *)p->slots};
        oe[i + 1] = oe[i] + belem_blocks(p->geo);
        oc[i + 1] = oc[i] + bnode_blocks(p->geo);
    }
    const size_t tb = (sizeof(BElem<T, T>) * n + 255) / 256 * 256, ob = sizeof(int) * (n + 1);
    FE_CHECK_HIP(hipMalloc(&B->dtab, tb + 2 * ob));
    char *d = static_cast<char *>(B->dtab);
    FE_CHECK_HIP(hipMemcpy(d, tab.data(), sizeof(BElem<T, T>) * n, hipMemcpyHostToDevice));
    FE_CHECK_HIP(hipMemcpy(d + tb, oe.data(), ob, hipMemcpyHostToDevice));
    FE_CHECK_HIP(hipMemcpy(d + tb + ob, oc.data(), ob, hipMemcpyHostToDevice));
    B->elem = BLaunch{d, reinterpret_cast<const int *>(d + tb), n, oe[n]};
    B->comb = BLaunch{d, reinterpret_cast<const int *>(d + tb + ob), n, oc[n]};
    return FE_OK;
}

}  // namespace

extern "C" {

int fe_jvp_batch_create(int n, fe_problem *const *probs, fe_prec prec, const void *const *x,
                        const double *const *gamma, const double *const *s_elem,
                        const void *const *v, void *const *jv, fe_batch **out)
{
    using namespace fe;
    if (!out || n < 1 || !probs || !x || !gamma || !s_elem || !v || !jv) {
        set_error("fe_jvp_batch_create: need n >= 1 and non-NULL arrays");
        return FE_EINVAL;
    }
    *out = nullptr;
    if (prec != FE_FP64 && prec != FE_FP32) {
        set_error("fe_jvp_batch_create: unknown precision");
        return FE_EINVAL;
    }
    std::vector<const fe_problem *> seen;
    for (int i = 0; i < n; ++i) {
        if (!probs[i] || !x[i] || !gamma[i] || !s_elem[i] || !v[i] || !jv[i]) {
            set_error("fe_jvp_batch_create: NULL entry " + std::to_string(i));
            return FE_EINVAL;
        }
        seen.push_back(probs[i]);
    }
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) {
        set_error("fe_jvp_batch_create: a problem appears twice (its work buffer would be shared)");
        return FE_EINVAL;
    }
    auto *B = new (std::nothrow) fe_batch();
    if (!B) return FE_ENOMEM;
    B->prec = prec;
    B->n = n;
    const int rc = prec == FE_FP64 ? jvp_batch_build<double>(B, n, probs, x, gamma, s_elem, v, jv)
                                   : jvp_batch_build<float>(B, n, probs, x, gamma, s_elem, v, jv);
    if (rc) {
        fe_jvp_batch_destroy(B);
        return rc;
    }
    *out = B;
    return FE_OK;
}

int fe_jvp_batch_run(fe_batch *B, hipStream_t stream)
{
    using namespace fe;
    if (!B) {
        set_error("fe_jvp_batch_run: NULL batch");
        return FE_EINVAL;
    }
    if (B->prec == FE_FP64) {
        FE_CHECK_HIP((blaunch_elem_jv<double, double>(B->elem, stream)));
        FE_CHECK_HIP((blaunch_combine_jv<double, double>(B->comb, stream)));
    } else {
        FE_CHECK_HIP((blaunch_elem_jv<float, float>(B->elem, stream)));
        FE_CHECK_HIP((blaunch_combine_jv<float, float>(B->comb, stream)));
    }
    return FE_OK;
}

int fe_jvp_batch_destroy(fe_batch *B)
{
    if (!B) return FE_OK;
    if (B->dtab) (void)hipFree(B->dtab);
    delete B;
    return FE_OK;
}

}  // extern "C"
