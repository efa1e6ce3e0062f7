// Matrix-free geometric multigrid preconditioner (host side).
//
// The paper preconditions flexible GMRES with geometric multigrid (Sec.
// "Solving the linear systems").  Here every level is a rediscretisation of the
// same stabilised operator on a grid with half the elements per direction:
// the design and source are averaged over the eight child elements, the
// linearisation state is injected from the coincident fine nodes, and the
// element kernels of the fine level evaluate J v on every level.  Smoothing is
// damped nodal block-Jacobi; the coarsest level is solved directly with a band
// LU factorisation of its assembled Jacobian (assembled on the GPU by 135
// probing products, one per (node colour mod 3^3, field)).  V-cycles run in
// FP64, or in FP32 when the Krylov operator is FP32.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fe_internal.h"
#include "fe_mg.h"

namespace fe {

hipError_t mg_coarsen_elem(int ncx, int ncy, int ncz, const double *f, double *c, hipStream_t st);
hipError_t mg_inject_state(int ncx, int ncy, int ncz, const double *f, double *c, hipStream_t st);
hipError_t mg_inject_mask(int ncx, int ncy, int ncz, const uint8_t *f, uint8_t *c, hipStream_t st);
template <typename T>
hipError_t mg_restrict(int ncx, int ncy, int ncz, const T *b, const T *t, const uint8_t *cmask, T *bc,
                       hipStream_t st);
template <typename T>
hipError_t mg_prolong_add(int nfx, int nfy, int nfz, const T *xc, const uint8_t *fmask, T *x,
                          hipStream_t st);
template <typename T>
hipError_t mg_smooth(const T *D, const T *b, const T *t, T *x, int64_t nn, T omega, bool transpose,
                     bool accumulate, hipStream_t st);

constexpr int64_t MG_MAX_COARSE_DOF = 2400;   // largest directly factored level
constexpr int64_t MG_TARGET_COARSE_DOF = 1500; // stop coarsening below this size

static void free_level(fe_problem *p, MgLevel &L, bool owned)
{
    if (owned) {
        dfree(p, L.nmask);
        dfree(p, L.gamma);
        dfree(p, L.s);
        dfree(p, L.x);
        dfree(p, L.x32);
        dfree(p, L.D);
        dfree(p, L.D32);
        dfree(p, L.slots);
        dfree(p, L.slots25);
    }
    dfree(p, L.b);
    dfree(p, L.xs);
    dfree(p, L.t);
    dfree(p, L.b32);
    dfree(p, L.xs32);
    dfree(p, L.t32);
}

void mg_free(Mg *mg)
{
    if (!mg) return;
    fe_problem *p = mg->owner;
    for (size_t l = 0; l < mg->lev.size(); ++l) free_level(p, mg->lev[l], l > 0);
    dfree(p, mg->probe);
    dfree(p, mg->probe_out);
    hfree(p, mg->hbuf);
    delete mg;
}

int mg_num_levels(const fe_grid &g)
{
    int nx = g.nx, ny = g.ny, nz = g.nz, n = 1;
    while (true) {
        const int64_t ndof = (int64_t)NF * (nx + 1) * (ny + 1) * (nz + 1);
        if (ndof <= MG_TARGET_COARSE_DOF) break;
        if (nx % 2 || ny % 2 || nz % 2 || nx < 4 || ny < 4 || nz < 4) break;
        nx /= 2;
        ny /= 2;
        nz /= 2;
        ++n;
    }
    const int64_t ndof = (int64_t)NF * (nx + 1) * (ny + 1) * (nz + 1);
    if (n < 2 || ndof > MG_MAX_COARSE_DOF) return 0;  // no usable hierarchy
    return n;
}

static int64_t r256(int64_t b) { return (b + 255) / 256 * 256; }

// Device bytes mg_create allocates for grid g (each allocation rounded up to 256 B).
int64_t mg_footprint_bytes(const fe_grid &g0, bool mixed)
{
    const int nl = mg_num_levels(g0);
    if (nl < 2) return 0;
    fe_grid g = g0;
    int64_t b = 0, ndof_c = 0, ne_c = 0;
    for (int l = 0; l < nl; ++l) {
        if (l > 0) {
            g.nx /= 2;
            g.ny /= 2;
            g.nz /= 2;
        }
        const int64_t nn = (int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1), ndof = NF * nn;
        const int64_t ne = (int64_t)g.nx * g.ny * g.nz;
        const int64_t nt = (int64_t)((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) * ((g.nz + TZ - 1) / TZ);
        if (l > 0) {
            b += r256(nn) + 2 * r256(8 * ne) + r256(8 * ndof) + r256(8 * 25 * nn);
            b += r256(nt * BOXN * NF * 8) + r256(nt * BOXN * 25 * 8);
            b += 2 * r256(8 * ndof);
            if (mixed) b += r256(4 * ndof) + r256(4 * 25 * nn) + 2 * r256(4 * ndof);
        } else if (mixed) {
            b += r256(4 * ndof);
        }
        b += r256(8 * ndof);
        if (mixed) b += r256(4 * ndof);
        ndof_c = ndof;
        ne_c = ne;
    }
    b += r256(8 * 1600 * ne_c) + r256(8 * 135 * ndof_c);
    return b;
}

// Allocate the hierarchy for problem p (levels >= 1 own their data).
int mg_create(fe_problem *p, bool mixed, Mg **out)
{
    *out = nullptr;
    const int nl = mg_num_levels(p->grid);
    if (nl < 2) {
        set_error("multigrid: the grid cannot be coarsened to a directly solvable level "
                  "(element counts must halve evenly down to <= 2400 coarse DOF)");
        return FE_EINVAL;
    }
    Mg *mg = new Mg();
    mg->owner = p;
    mg->mixed = mixed;
    mg->lev.resize(nl);
    hipError_t e = hipSuccess;
    fe_grid g = p->grid;
    for (int l = 0; l < nl; ++l) {
        MgLevel &L = mg->lev[l];
        if (l > 0) {
            g.nx /= 2;
            g.ny /= 2;
            g.nz /= 2;
            g.h *= 2.0;
        }
        L.grid = g;
        L.geo = make_geo(g, p->phys);
        L.nn = n_nodes(L.geo);
        L.ne = n_elem(L.geo);
        L.ndof = NF * L.nn;
        const size_t nb = sizeof(double) * L.ndof;
        if (l > 0) {
            if (e == hipSuccess) e = dalloc(p, &L.nmask, L.nn);
            if (e == hipSuccess) e = dalloc(p, &L.gamma, sizeof(double) * L.ne);
            if (e == hipSuccess) e = dalloc(p, &L.s, sizeof(double) * L.ne);
            if (e == hipSuccess) e = dalloc(p, &L.x, nb);
            if (e == hipSuccess) e = dalloc(p, &L.D, sizeof(double) * 25 * L.nn);
            if (e == hipSuccess) e = dalloc(p, &L.slots, (size_t)n_tiles(L.geo) * BOXN * NF * sizeof(double));
            if (e == hipSuccess) e = dalloc(p, &L.slots25, (size_t)n_tiles(L.geo) * BOXN * 25 * sizeof(double));
            if (e == hipSuccess && mixed) e = dalloc(p, &L.x32, sizeof(float) * L.ndof);
            if (e == hipSuccess && mixed) e = dalloc(p, &L.D32, sizeof(float) * 25 * L.nn);
            if (e == hipSuccess) e = dalloc(p, &L.b, nb);
            if (e == hipSuccess) e = dalloc(p, &L.xs, nb);
            if (e == hipSuccess && mixed) e = dalloc(p, &L.b32, sizeof(float) * L.ndof);
            if (e == hipSuccess && mixed) e = dalloc(p, &L.xs32, sizeof(float) * L.ndof);
        } else if (mixed) {
            if (e == hipSuccess) e = dalloc(p, &L.b32, sizeof(float) * L.ndof);  // cast of the Krylov vector
        }
        if (e == hipSuccess) e = dalloc(p, &L.t, nb);
        if (e == hipSuccess && mixed) e = dalloc(p, &L.t32, sizeof(float) * L.ndof);
    }
    const MgLevel &C = mg->lev.back();
    mg->nc = C.ndof;
    if (e == hipSuccess) e = dalloc(p, &mg->probe, sizeof(double) * 1600 * C.ne);  // element Jacobians
    if (e == hipSuccess) e = dalloc(p, &mg->probe_out, sizeof(double) * 135 * C.ndof);
    if (e == hipSuccess) e = halloc(p, &mg->hbuf, sizeof(double) * 135 * C.ndof);
    if (e != hipSuccess) {
        mg_free(mg);
        return hip_fail(e, "hipMalloc (multigrid)");
    }
    const int bw = (int)(NF * (1 + (C.grid.nx + 1) + (int64_t)(C.grid.nx + 1) * (C.grid.ny + 1)) + NF - 1);
    mg->kl = mg->ku = bw;
    mg->A.assign((size_t)C.ndof * C.ndof, 0.0);
    mg->piv.assign(C.ndof, 0);
    mg->Lc.assign((size_t)C.ndof * bw, 0.0);
    mg->Uc.assign((size_t)C.ndof * 2 * bw, 0.0);
    mg->hb.assign(C.ndof + 2 * bw, 0.0);  // 2 bw entries of scratch, then the vector
    *out = mg;
    return FE_OK;
}

// Coarse design and source, once per solve (the design is fixed during it).
int mg_set_design(Mg *mg, fe_problem *p, const double *gamma, const double *s, hipStream_t st)
{
    mg->lev[0].gamma = const_cast<double *>(gamma);
    mg->lev[0].s = const_cast<double *>(s);
    mg->lev[0].nmask = p->nmask;
    mg->lev[0].slots = p->slots;
    for (auto &L : mg->lev) L.geo = make_geo(L.grid, p->phys);  // parameters may have changed
    for (size_t l = 1; l < mg->lev.size(); ++l) {
        MgLevel &C = mg->lev[l], &F = mg->lev[l - 1];
        FE_CHECK_HIP(mg_coarsen_elem(C.grid.nx, C.grid.ny, C.grid.nz, F.gamma, C.gamma, st));
        FE_CHECK_HIP(mg_coarsen_elem(C.grid.nx, C.grid.ny, C.grid.nz, F.s, C.s, st));
        FE_CHECK_HIP(mg_inject_mask(C.grid.nx, C.grid.ny, C.grid.nz, F.nmask, C.nmask, st));
    }
    return FE_OK;
}

// Band LU with partial pivoting of the dense-stored coarsest matrix.
static int band_lu(Mg *mg)
{
    const int64_t n = mg->nc;
    const int kl = mg->kl, ku = mg->ku;
    double *A = mg->A.data();
    for (int64_t k = 0; k < n; ++k) {
        const int64_t iend = std::min<int64_t>(n - 1, k + kl);
        int64_t p = k;
        double best = std::fabs(A[k * n + k]);
        for (int64_t i = k + 1; i <= iend; ++i)
            if (std::fabs(A[i * n + k]) > best) {
                best = std::fabs(A[i * n + k]);
                p = i;
            }
        mg->piv[k] = (int)p;
        if (best == 0.0 || !std::isfinite(best)) {
            set_error("multigrid: singular or non-finite coarsest-level matrix");
            return FE_ENAN;
        }
        const int64_t jend = std::min<int64_t>(n - 1, k + kl + ku);
        if (p != k)
            for (int64_t j = k; j <= jend; ++j) std::swap(A[k * n + j], A[p * n + j]);
        const double inv = 1.0 / A[k * n + k];
        for (int64_t i = k + 1; i <= iend; ++i) {
            const double l = A[i * n + k] * inv;
            A[i * n + k] = l;
            mg->Lc[k * kl + (i - k - 1)] = l;
            if (l != 0.0)
                for (int64_t j = k + 1; j <= jend; ++j) A[i * n + j] -= l * A[k * n + j];
        }
        for (int64_t i = iend + 1; i <= k + kl; ++i) mg->Lc[k * kl + (i - k - 1)] = 0.0;
    }
    // U by columns for the back substitution: Uc[k w + t] = U(k - w + t, k), w = kl + ku
    const int64_t w = kl + ku;
    for (int64_t k = 0; k < n; ++k)
        for (int64_t t = 0; t < w; ++t) {
            const int64_t r = k - w + t;
            mg->Uc[k * w + t] = r >= 0 ? A[r * n + k] : 0.0;
        }
    return FE_OK;
}

// b: the right-hand side on entry, the solution on exit; it is preceded by
// kl + ku entries of scratch (the back substitution's column updates run into
// them instead of being clipped).  Both sweeps of the forward solve are
// contiguous multiply-subtract loops over a column of L or U.
static void band_solve(const Mg *mg, double *b, bool transpose)
{
    const int64_t n = mg->nc;
    const int kl = mg->kl, ku = mg->ku;
    const double *A = mg->A.data();
    if (!transpose) {
        const double *__restrict__ Lc = mg->Lc.data();  // multipliers of column k, contiguous
        for (int64_t k = 0; k < n; ++k) {
            const int64_t p = mg->piv[k];
            if (p != k) std::swap(b[k], b[p]);
            const int64_t cnt = std::min<int64_t>(n - 1, k + kl) - k;
            const double bk = b[k];
            const double *__restrict__ l = Lc + k * kl;
            double *__restrict__ y = b + k + 1;
            for (int64_t q = 0; q < cnt; ++q) y[q] -= l[q] * bk;
        }
        const int64_t w = kl + ku;
        for (int64_t t = 1; t <= w; ++t) b[-t] = 0.0;
        for (int64_t k = n - 1; k >= 0; --k) {
            const double xk = b[k] / A[k * n + k];
            b[k] = xk;
            const double *__restrict__ u = mg->Uc.data() + k * w;
            double *__restrict__ y = b + k - w;
            for (int64_t t = 0; t < w; ++t) y[t] -= u[t] * xk;
        }
    } else {
        // A^T x = b with A = P^T L U: U^T y = b, then L^T and the swaps in reverse
        for (int64_t k = 0; k < n; ++k) {
            const int64_t j0 = std::max<int64_t>(0, k - kl - ku);
            double s = b[k];
            for (int64_t j = j0; j < k; ++j) s -= A[j * n + k] * b[j];
            b[k] = s / A[k * n + k];
        }
        const double *Lc = mg->Lc.data();
        for (int64_t k = n - 1; k >= 0; --k) {
            const int64_t cnt = std::min<int64_t>(n - 1, k + kl) - k;
            double s = b[k];
            for (int64_t q = 0; q < cnt; ++q) s -= Lc[k * kl + q] * b[k + 1 + q];
            b[k] = s;
            const int64_t p = mg->piv[k];
            if (p != k) std::swap(b[k], b[p]);
        }
    }
}

// Per Newton step: linearisation states and block diagonals on every level,
// FP32 copies in mixed mode, and the coarsest-level factorisation.
int mg_setup(Mg *mg, fe_problem *p, const double *x, const double *D0, const float *D032,
             const float *x032, hipStream_t st)
{
    MgLevel &L0 = mg->lev[0];
    L0.x = const_cast<double *>(x);
    L0.D = const_cast<double *>(D0);
    L0.D32 = const_cast<float *>(D032);
    L0.x32 = const_cast<float *>(x032);
    const int nl = (int)mg->lev.size();
    for (int l = 1; l < nl; ++l) {
        MgLevel &C = mg->lev[l], &F = mg->lev[l - 1];
        FE_CHECK_HIP(mg_inject_state(C.grid.nx, C.grid.ny, C.grid.nz, F.x, C.x, st));
        if (l < nl - 1) {
            FE_CHECK_HIP(launch_blockdiag(C.geo, C.x, C.gamma, C.s, C.nmask, C.D, C.slots25, st));
            FE_CHECK_HIP(launch_invert_blocks(C.D, mg->mixed ? C.D32 : nullptr, C.nn, st));
            if (mg->mixed) FE_CHECK_HIP((launch_cast<double, float>(C.x, C.x32, C.ndof, st)));
        }
    }
    // coarsest level: the 135 probing products J p_(colour,field) in FP64, from
    // its element Jacobians (two launches)
    MgLevel &C = mg->lev.back();
    FE_CHECK_HIP(launch_probe_products(C.geo, C.x, C.gamma, C.s, C.nmask, mg->probe,
                                       mg->probe_out, st));
    FE_CHECK_HIP(hipMemcpyAsync(mg->hbuf, mg->probe_out, sizeof(double) * 135 * C.ndof,
                                hipMemcpyDeviceToHost, st));
    FE_CHECK_HIP(hipStreamSynchronize(st));
    assemble_from_probes(C.grid, mg->hbuf, mg->A.data());
    return band_lu(mg);
}

// Dense row-major J from the 135 colour-by-field probing products: entry
// (N g, M f) is row N g of product (colour(M), f), M within one node of N.
void assemble_from_probes(const fe_grid &grid, const double *probe, double *A)
{
    const int nx = grid.nx, ny = grid.ny, nz = grid.nz;
    const int64_t n = NF * (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    std::fill(A, A + n * n, 0.0);
    for (int K = 0; K <= nz; ++K)
        for (int J = 0; J <= ny; ++J)
            for (int I = 0; I <= nx; ++I) {
                const int64_t N = I + (int64_t)(nx + 1) * (J + (int64_t)(ny + 1) * K);
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int i = I + dx, j = J + dy, k = K + dz;
                            if (i < 0 || j < 0 || k < 0 || i > nx || j > ny || k > nz) continue;
                            const int64_t M = i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k);
                            const int col = (i % 3) + 3 * (j % 3) + 9 * (k % 3);
                            for (int g = 0; g < NF; ++g)
                                for (int f = 0; f < NF; ++f)
                                    A[(NF * N + g) * n + NF * M + f] =
                                        probe[(int64_t)(NF * col + f) * n + NF * N + g];
                        }
            }
}

template <typename T>
static T *vecT(MgLevel &L, int which);
template <>
double *vecT<double>(MgLevel &L, int which) { return which == 0 ? L.b : which == 1 ? L.xs : L.t; }
template <>
float *vecT<float>(MgLevel &L, int which) { return which == 0 ? L.b32 : which == 1 ? L.xs32 : L.t32; }
template <typename T>
static const T *stateT(const MgLevel &L);
template <>
const double *stateT<double>(const MgLevel &L) { return L.x; }
template <>
const float *stateT<float>(const MgLevel &L) { return L.x32; }
template <typename T>
static const T *blocksT(const MgLevel &L);
template <>
const double *blocksT<double>(const MgLevel &L) { return L.D; }
template <>
const float *blocksT<float>(const MgLevel &L) { return L.D32; }

template <typename T>
static hipError_t op(const MgLevel &L, const T *v, T *out, bool tr, hipStream_t st)
{
    return launch_elem<T, T>(tr ? OP_JTV : OP_JV, L.geo, stateT<T>(L), v, L.gamma, L.s, L.nmask, out,
                             (T *)L.slots, st);
}

template <typename T>
static int coarse_solve(Mg *mg, MgLevel &C, const T *b, T *x, bool tr, hipStream_t st)
{
    const int64_t n = C.ndof;
    T *h = reinterpret_cast<T *>(mg->hbuf);
    FE_CHECK_HIP(hipMemcpyAsync(h, b, sizeof(T) * n, hipMemcpyDeviceToHost, st));
    FE_CHECK_HIP(hipStreamSynchronize(st));
    double *hb = mg->hb.data() + (mg->kl + mg->ku);
    for (int64_t i = 0; i < n; ++i) hb[i] = (double)h[i];
    band_solve(mg, hb, tr);
    for (int64_t i = 0; i < n; ++i) h[i] = (T)hb[i];
    FE_CHECK_HIP(hipMemcpyAsync(x, h, sizeof(T) * n, hipMemcpyHostToDevice, st));
    return FE_OK;
}

template <typename T>
static int vcycle(Mg *mg, int l, const T *b, T *x, bool tr, hipStream_t st)
{
    MgLevel &L = mg->lev[l];
    const int nl = (int)mg->lev.size();
    if (l == nl - 1) return coarse_solve<T>(mg, L, b, x, tr, st);
    const T om = (T)mg->omega;
    const T *D = blocksT<T>(L);
    T *t = vecT<T>(L, 2);
    FE_CHECK_HIP(mg_smooth<T>(D, b, nullptr, x, L.nn, om, tr, false, st));
    for (int it = 1; it < mg->nu1; ++it)
        FE_CHECK_HIP(launch_elem_smooth<T>(tr, L.geo, stateT<T>(L), x, L.gamma, L.s, L.nmask, t,
                                           (T *)L.slots, D, b, om, st));
    MgLevel &C = mg->lev[l + 1];
    FE_CHECK_HIP(op<T>(L, x, t, tr, st));
    T *bc = vecT<T>(C, 0), *xc = vecT<T>(C, 1);
    FE_CHECK_HIP(mg_restrict<T>(C.grid.nx, C.grid.ny, C.grid.nz, b, t, C.nmask, bc, st));
    int rc = vcycle<T>(mg, l + 1, bc, xc, tr, st);
    if (rc) return rc;
    FE_CHECK_HIP(mg_prolong_add<T>(L.grid.nx, L.grid.ny, L.grid.nz, xc, L.nmask, x, st));
    for (int it = 0; it < mg->nu2; ++it)
        FE_CHECK_HIP(launch_elem_smooth<T>(tr, L.geo, stateT<T>(L), x, L.gamma, L.s, L.nmask, t,
                                           (T *)L.slots, D, b, om, st));
    return FE_OK;
}

int mg_apply64(Mg *mg, const double *v, double *z, bool tr, hipStream_t st)
{
    return vcycle<double>(mg, 0, v, z, tr, st);
}

int mg_apply32(Mg *mg, const double *v, float *z, bool tr, hipStream_t st)
{
    MgLevel &L0 = mg->lev[0];
    FE_CHECK_HIP((launch_cast<double, float>(v, L0.b32, L0.ndof, st)));
    return vcycle<float>(mg, 0, L0.b32, z, tr, st);
}

}  // namespace fe
