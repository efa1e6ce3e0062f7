// Matrix-free geometric multigrid preconditioner (host side).
//
// The paper preconditions flexible GMRES with geometric multigrid (Sec.
// "Solving the linear systems").  Here every level is a rediscretisation of the
// same stabilised operator on a grid with half the elements per direction:
// the design and source are averaged over the eight child elements, the
// linearisation state is injected from the coincident fine nodes, and the
// element kernels of the fine level evaluate J v on every level.  Smoothing is
// damped nodal block-Jacobi; small levels apply their operator as an assembled
// 27-point block stencil (from element Jacobians, once per Newton step), since
// the element pass costs the same latency however few tiles a grid has.  The
// coarsest level is solved directly: its Jacobian is assembled from 135
// probing products (one per (node colour mod 3^3, field)), condensed to the
// DOFs that are not prescribed (prescribed rows are identity rows and
// prescribed columns are zero, so they drop out exactly), factorised by band
// LU on the host, and inverted explicitly on the GPU from the factors, so that
// each V-cycle's coarse solve is one matrix-vector product on the device.
// V-cycles run in FP64, or in FP32 when the Krylov operator is FP32.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fe_internal.h"
#include "fe_mg.h"

namespace fe {

hipError_t mg_coarsen_elem(const fe_grid &c, const fe_grid &f, const double *fv, double *cv,
                          hipStream_t st);
hipError_t mg_inject_state(const fe_grid &c, const fe_grid &f, const double *fv, double *cv,
                           hipStream_t st);
hipError_t mg_inject_mask(const fe_grid &c, const fe_grid &f, const uint8_t *fv, uint8_t *cv,
                          hipStream_t st);
template <typename T>
hipError_t mg_restrict(const fe_grid &c, const fe_grid &f, const T *b, const T *t,
                       const uint8_t *cmask, T *bc, hipStream_t st);
template <typename T>
hipError_t mg_restrict_smooth(const fe_grid &c, const fe_grid &f, const T *b, const T *t,
                              const uint8_t *cmask, T *bc, const T *Dc, T *xc, T omega,
                              bool transpose, hipStream_t st);
template <typename T>
hipError_t mg_prolong_add(const fe_grid &f, const fe_grid &c, const T *xc, const uint8_t *fmask,
                          T *x, hipStream_t st);
template <typename T>
hipError_t mg_smooth(const T *D, const T *b, const T *t, T *x, int64_t nn, T omega, bool transpose,
                     bool accumulate, hipStream_t st);
template <typename T>
hipError_t mg_stencil_apply(int nx, int ny, int nz, const T *S, const T *v, T *out, bool transpose,
                            hipStream_t st);
hipError_t mg_stencil_diag(int64_t nn, const double *S, double *D, hipStream_t st);
hipError_t mg_coarse_inverse(int n, int kl, int ku, const double *Lc, const double *Uc,
                             const double *Ud, const int *piv, double *X, hipStream_t st);
template <typename T>
hipError_t mg_coarse_apply(int n, int m, const double *X, const int *fidx, const int *pos, const T *b,
                           T *x, double *P, bool transpose, hipStream_t st);
template <typename T>
hipError_t mg_stencil_smooth(int nx, int ny, int nz, const T *S, const T *D, const T *b, const T *xin,
                             T *xout, T omega, bool transpose, hipStream_t st);
hipError_t mg_smooth0_cast(const float *D, const double *v, float *b32, float *x, int64_t nn,
                           float omega, bool transpose, hipStream_t st);
template <typename T>
hipError_t mg_copy(const T *a, T *b, int64_t n, hipStream_t st);

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
    dfree(p, L.S);
    dfree(p, L.S32);
    dfree(p, L.xa);
    dfree(p, L.xa32);
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
    dfree(p, mg->dfac);
    dfree(p, mg->dpiv);
    dfree(p, mg->dmap);
    dfree(p, mg->Xinv);
    dfree(p, mg->cpart);
    hfree(p, mg->hbuf);
    hfree(p, mg->hfac);
    hfree(p, mg->hpiv);
    hfree(p, mg->hmask);
    hfree(p, mg->hmap);
    if (mg->probe_ready) (void)hipEventDestroy(mg->probe_ready);
    delete mg;
}

int64_t mg_asm_nodes(int opt) { return opt < 0 ? MG_ASM_NODES_DEFAULT : (int64_t)opt; }

// Next coarser grid: elements of twice the edge, ceil(n / 2) per direction.  An
// odd fine count leaves the last coarse layer half outside the fine grid; its
// nodes past the end take their values from the fine boundary nodes.
static fe_grid coarser(fe_grid g)
{
    g.nx = (g.nx + 1) / 2;
    g.ny = (g.ny + 1) / 2;
    g.nz = (g.nz + 1) / 2;
    g.h *= 2.0;
    return g;
}

// Levels while the coarse grids stay nested (every count even) or, with pad,
// also through odd counts; 0 when that gives no usable hierarchy.
static int count_levels(fe_grid g, bool pad)
{
    int n = 1;
    while (true) {
        const int64_t ndof = (int64_t)NF * (g.nx + 1) * (g.ny + 1) * (g.nz + 1);
        if (ndof <= MG_TARGET_COARSE_DOF) break;
        if (g.nx < 4 || g.ny < 4 || g.nz < 4) break;
        if (!pad && (g.nx % 2 || g.ny % 2 || g.nz % 2)) break;
        g = coarser(g);
        ++n;
    }
    const int64_t ndof = (int64_t)NF * (g.nx + 1) * (g.ny + 1) * (g.nz + 1);
    if (n < 2 || ndof > MG_MAX_COARSE_DOF) return 0;
    return n;
}

// Nested levels where they give a hierarchy; otherwise (odd counts before the
// coarse problem is small enough) padded ones.
int mg_num_levels(const fe_grid &g)
{
    const int n = count_levels(g, false);
    return n ? n : count_levels(g, true);
}

static int64_t r256(int64_t b) { return (b + 255) / 256 * 256; }

// Half bandwidth of the coarsest matrix in lexicographic node order, NF DOF per node.
static int64_t coarse_band(const fe_grid &c)
{
    return NF * (1 + (c.nx + 1) + (int64_t)(c.nx + 1) * (c.ny + 1)) + NF - 1;
}

// Device bytes mg_create allocates for grid g (each allocation rounded up to 256 B).
int64_t mg_footprint_bytes(const fe_grid &g0, bool mixed, int64_t asm_nodes)
{
    const int nl = mg_num_levels(g0);
    if (nl < 2) return 0;
    fe_grid g = g0;
    int64_t b = 0, ndof_c = 0, ne_c = 0, ne_je = 0;
    for (int l = 0; l < nl; ++l) {
        if (l > 0) g = coarser(g);
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
        if (l < nl - 1 && nn <= asm_nodes) {
            b += r256(8 * 675 * nn) + r256(8 * ndof);
            if (mixed) b += r256(4 * 675 * nn) + r256(4 * ndof);
            ne_je = std::max(ne_je, ne);
        }
        ndof_c = ndof;
        ne_c = ne;
    }
    b += r256(8 * 1600 * std::max(ne_c, ne_je)) + r256(8 * 135 * ndof_c);
    const int64_t bw = coarse_band(g);
    b += r256(8 * ndof_c * (3 * bw + 1)) + r256(4 * ndof_c) + r256(8 * ndof_c) + r256(8 * ndof_c * ndof_c);
    b += r256(8 * ((ndof_c + 63) / 64) * ndof_c);
    return b;
}

// Allocate the hierarchy for problem p (levels >= 1 own their data).
int mg_create(fe_problem *p, bool mixed, int64_t asm_nodes, Mg **out)
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
    mg->asm_nodes = asm_nodes;
    mg->lev.resize(nl);
    hipError_t e = hipSuccess;
    fe_grid g = p->grid;
    for (int l = 0; l < nl; ++l) {
        MgLevel &L = mg->lev[l];
        if (l > 0) g = coarser(g);
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
        L.assembled = l < nl - 1 && L.nn <= asm_nodes;
        if (L.assembled) {
            if (e == hipSuccess) e = dalloc(p, &L.S, sizeof(double) * 675 * L.nn);
            if (e == hipSuccess && mixed) e = dalloc(p, &L.S32, sizeof(float) * 675 * L.nn);
            if (e == hipSuccess) e = dalloc(p, &L.xa, nb);
            if (e == hipSuccess && mixed) e = dalloc(p, &L.xa32, sizeof(float) * L.ndof);
        }
    }
    const MgLevel &C = mg->lev.back();
    mg->nc = C.ndof;
    int64_t ne_je = C.ne;
    for (const MgLevel &L : mg->lev)
        if (L.assembled) ne_je = std::max(ne_je, L.ne);
    if (e == hipSuccess) e = dalloc(p, &mg->probe, sizeof(double) * 1600 * ne_je);  // element Jacobians
    if (e == hipSuccess) e = dalloc(p, &mg->probe_out, sizeof(double) * 135 * C.ndof);
    if (e == hipSuccess) e = halloc(p, &mg->hbuf, sizeof(double) * 135 * C.ndof);
    // sized for the full matrix: condensing never widens the band
    const int bw = (int)coarse_band(C.grid);
    mg->bw = bw;
    const size_t nfac = (size_t)C.ndof * (3 * bw + 1);
    if (e == hipSuccess) e = halloc(p, &mg->hfac, sizeof(double) * nfac);
    if (e == hipSuccess) e = halloc(p, &mg->hpiv, sizeof(int) * C.ndof);
    if (e == hipSuccess) e = halloc(p, &mg->hmask, C.nn);
    if (e == hipSuccess) e = halloc(p, &mg->hmap, sizeof(int) * 2 * C.ndof);
    if (e == hipSuccess) e = dalloc(p, &mg->dfac, sizeof(double) * nfac);
    if (e == hipSuccess) e = dalloc(p, &mg->dpiv, sizeof(int) * C.ndof);
    if (e == hipSuccess) e = dalloc(p, &mg->dmap, sizeof(int) * 2 * C.ndof);
    if (e == hipSuccess) e = dalloc(p, &mg->Xinv, sizeof(double) * C.ndof * C.ndof);
    if (e == hipSuccess) e = dalloc(p, &mg->cpart, sizeof(double) * ((C.ndof + 63) / 64) * C.ndof);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&mg->probe_ready, hipEventDisableTiming);
    if (e != hipSuccess) {
        mg_free(mg);
        return hip_fail(e, "hipMalloc (multigrid)");
    }
    mg->A.assign((size_t)C.ndof * C.ndof, 0.0);
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
        FE_CHECK_HIP(mg_coarsen_elem(C.grid, F.grid, F.gamma, C.gamma, st));
        FE_CHECK_HIP(mg_coarsen_elem(C.grid, F.grid, F.s, C.s, st));
        FE_CHECK_HIP(mg_inject_mask(C.grid, F.grid, F.nmask, C.nmask, st));
    }
    mg->coarse_ready = false;  // the coarsest matrix depends on the design
    return FE_OK;
}

// Index maps of the coarsest level's free DOFs from its node mask (free DOFs
// keep their lexicographic order), and the half bandwidths of the condensed
// matrix: the largest index distance between two free DOFs of nodes at most one
// node apart in each direction.
static void condense_coarse(Mg *mg, const fe_grid &grid)
{
    const int64_t n = mg->nc;
    int *fidx = mg->hmap, *pos = mg->hmap + n;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if ((mg->hmask[i / NF] >> (i % NF)) & 1) {
            pos[i] = -1;
        } else {
            pos[i] = (int)m;
            fidx[m++] = (int)i;
        }
    }
    mg->nf = m;
    const int nx = grid.nx, ny = grid.ny, nz = grid.nz;
    int64_t lo = 0, hi = 0;
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
                            for (int g = 0; g < NF; ++g) {
                                const int r = pos[NF * N + g];
                                if (r < 0) continue;
                                for (int f = 0; f < NF; ++f) {
                                    const int c = pos[NF * M + f];
                                    if (c < 0) continue;
                                    lo = std::max<int64_t>(lo, r - c);
                                    hi = std::max<int64_t>(hi, c - r);
                                }
                            }
                        }
            }
    // at least one sub- and super-diagonal (zero ones where the matrix has none)
    mg->kl = (int)std::min<int64_t>(std::max<int64_t>(lo, 1), mg->bw);
    mg->ku = (int)std::min<int64_t>(std::max<int64_t>(hi, 1), mg->bw);
}

// The coarsest matrix restricted to its free DOFs, dense row-major nf x nf, from
// the 135 colour-by-field probing products: entry (pos[N g], pos[M f]) is row
// N g of product (colour(M), f), M within one node of N, both DOFs free.
static void assemble_free_from_probes(const fe_grid &grid, const double *probe, const int *pos,
                                      int64_t m, double *A)
{
    const int nx = grid.nx, ny = grid.ny, nz = grid.nz;
    const int64_t n = NF * (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    std::fill(A, A + m * m, 0.0);
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
                            for (int g = 0; g < NF; ++g) {
                                const int r = pos[NF * N + g];
                                if (r < 0) continue;
                                for (int f = 0; f < NF; ++f) {
                                    const int c = pos[NF * M + f];
                                    if (c >= 0) A[r * m + c] = probe[(int64_t)(NF * col + f) * n + NF * N + g];
                                }
                            }
                        }
            }
}

// Band LU with partial pivoting of the dense-stored condensed coarsest matrix
// (nf x nf); the factors go to the pinned buffers in the layout the device
// inverse reads.
static int band_lu(Mg *mg)
{
    const int64_t n = mg->nf;
    const int kl = mg->kl, ku = mg->ku;
    const int64_t w = kl + ku;
    double *A = mg->A.data();
    double *Lc = mg->hfac, *Uc = Lc + n * kl, *Ud = Uc + n * w;
    int *piv = mg->hpiv;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t iend = std::min<int64_t>(n - 1, k + kl);
        int64_t p = k;
        double best = std::fabs(A[k * n + k]);
        for (int64_t i = k + 1; i <= iend; ++i)
            if (std::fabs(A[i * n + k]) > best) {
                best = std::fabs(A[i * n + k]);
                p = i;
            }
        piv[k] = (int)p;
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
            Lc[k * kl + (i - k - 1)] = l;
            if (l != 0.0)
                for (int64_t j = k + 1; j <= jend; ++j) A[i * n + j] -= l * A[k * n + j];
        }
        for (int64_t i = iend + 1; i <= k + kl; ++i) Lc[k * kl + (i - k - 1)] = 0.0;
    }
    // U by columns: Uc[k w + t] = U(k - w + t, k), and its diagonal
    for (int64_t k = 0; k < n; ++k) {
        for (int64_t t = 0; t < w; ++t) {
            const int64_t r = k - w + t;
            Uc[k * w + t] = r >= 0 ? A[r * n + k] : 0.0;
        }
        Ud[k] = A[k * n + k];
    }
    return FE_OK;
}

// Per Newton step, in two calls around the caller's own fine-level set-up:
// mg_setup_begin injects the linearisation state into every level and starts
// the coarsest level's probing products and their copy to the host;
// mg_setup_finish builds the block diagonals (and FP32 copies in mixed mode)
// and assembled stencils of the other levels, then factorises the coarsest
// level on the host (overlapping that GPU work) and inverts it on the device.
int mg_setup_begin(Mg *mg, fe_problem *p, const double *x, hipStream_t st)
{
    (void)p;
    mg->lev[0].x = const_cast<double *>(x);
    const int nl = (int)mg->lev.size();
    for (int l = 1; l < nl; ++l) {
        MgLevel &C = mg->lev[l], &F = mg->lev[l - 1];
        FE_CHECK_HIP(mg_inject_state(C.grid, F.grid, F.x, C.x, st));
    }
    // with a kept factorisation the coarsest level is not probed again
    mg->skip_coarse = mg->reuse_coarse && mg->coarse_ready;
    if (mg->skip_coarse) return FE_OK;
    // the 135 probing products J p_(colour,field) in FP64 from the coarsest
    // level's element Jacobians (two launches), copied to the host
    MgLevel &C = mg->lev.back();
    FE_CHECK_HIP(launch_probe_products(C.geo, C.x, C.gamma, C.s, C.nmask, mg->probe,
                                       mg->probe_out, st));
    FE_CHECK_HIP(hipMemcpyAsync(mg->hbuf, mg->probe_out, sizeof(double) * 135 * C.ndof,
                                hipMemcpyDeviceToHost, st));
    FE_CHECK_HIP(hipMemcpyAsync(mg->hmask, C.nmask, C.nn, hipMemcpyDeviceToHost, st));
    FE_CHECK_HIP(hipEventRecord(mg->probe_ready, st));
    return FE_OK;
}

int mg_setup_finish(Mg *mg, fe_problem *p, const double *D0, const float *D032, const float *x032,
                    hipStream_t st)
{
    (void)p;
    MgLevel &L0 = mg->lev[0];
    L0.D = const_cast<double *>(D0);
    L0.D32 = const_cast<float *>(D032);
    L0.x32 = const_cast<float *>(x032);
    const int nl = (int)mg->lev.size();
    MgLevel &C = mg->lev.back();
    // a mixed-precision Newton step (FP32 state given) smooths with FP32 blocks
    // only, formed and inverted in FP32; otherwise (FP64 solves, the adjoint)
    // the blocks are FP64, with an FP32 copy in a mixed hierarchy
    const bool blocks32 = x032 != nullptr;
    for (int l = 1; l < nl - 1; ++l) {
        MgLevel &L = mg->lev[l];
        if (mg->mixed) FE_CHECK_HIP((launch_cast<double, float>(L.x, L.x32, L.ndof, st)));
        if (L.assembled) continue;
        if (blocks32) {
            FE_CHECK_HIP((launch_blockdiag<float>(L.geo, L.x32, L.gamma, L.s, L.nmask, L.D32,
                                                  reinterpret_cast<float *>(L.slots25), st)));
            FE_CHECK_HIP(launch_invert_blocks32(L.D32, L.nn, st));
        } else {
            FE_CHECK_HIP((launch_blockdiag<double>(L.geo, L.x, L.gamma, L.s, L.nmask, L.D,
                                                   L.slots25, st)));
            FE_CHECK_HIP(launch_invert_blocks(L.D, mg->mixed ? L.D32 : nullptr, L.nn, st));
        }
    }
    // assembled levels: element Jacobians, then the 27-point block stencil, whose
    // centre blocks are the smoother's diagonal blocks (below the finest level,
    // whose blocks the caller provides)
    for (int l = 0; l < nl - 1; ++l) {
        MgLevel &L = mg->lev[l];
        if (!L.assembled) continue;
        FE_CHECK_HIP(launch_stencil_assemble(L.geo, L.x, L.gamma, L.s, L.nmask, mg->probe, L.S, st));
        if (mg->mixed) FE_CHECK_HIP((launch_cast<double, float>(L.S, L.S32, 675 * L.nn, st)));
        if (l > 0) {
            FE_CHECK_HIP(mg_stencil_diag(L.nn, L.S, L.D, st));
            FE_CHECK_HIP(launch_invert_blocks(L.D, mg->mixed ? L.D32 : nullptr, L.nn, st));
        }
    }
    if (mg->skip_coarse) return FE_OK;  // the kept factorisation serves this step
    // (the event also orders the previous set-up's copy out of hfac before the
    // factorisation below rewrites it)
    FE_CHECK_HIP(hipEventSynchronize(mg->probe_ready));
    condense_coarse(mg, C.grid);
    assemble_free_from_probes(C.grid, mg->hbuf, mg->hmap + mg->nc, mg->nf, mg->A.data());
    int rc = band_lu(mg);
    if (rc) return rc;
    // the factors and index maps to the device, then the inverse column by column
    const int64_t n = mg->nf, w = mg->kl + mg->ku;
    if (n > 0) {
        FE_CHECK_HIP(hipMemcpyAsync(mg->dfac, mg->hfac, sizeof(double) * n * (mg->kl + w + 1),
                                    hipMemcpyHostToDevice, st));
        FE_CHECK_HIP(hipMemcpyAsync(mg->dpiv, mg->hpiv, sizeof(int) * n, hipMemcpyHostToDevice, st));
    }
    FE_CHECK_HIP(hipMemcpyAsync(mg->dmap, mg->hmap, sizeof(int) * 2 * mg->nc, hipMemcpyHostToDevice, st));
    const double *Lc = mg->dfac, *Uc = Lc + n * mg->kl, *Ud = Uc + n * w;
    if (n > 0) FE_CHECK_HIP(mg_coarse_inverse((int)n, mg->kl, mg->ku, Lc, Uc, Ud, mg->dpiv, mg->Xinv, st));
    mg->coarse_ready = true;
    return FE_OK;
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
static const T *stencilT(const MgLevel &L);
template <>
const double *stencilT<double>(const MgLevel &L) { return L.S; }
template <>
const float *stencilT<float>(const MgLevel &L) { return L.S32; }

template <typename T>
static hipError_t op(const MgLevel &L, const T *v, T *out, bool tr, hipStream_t st)
{
    if (L.assembled)
        return mg_stencil_apply<T>(L.grid.nx, L.grid.ny, L.grid.nz, stencilT<T>(L), v, out, tr, st);
    return launch_elem<T, T>(tr ? OP_JTV : OP_JV, L.geo, stateT<T>(L), v, L.gamma, L.s, L.nmask, out,
                             (T *)L.slots, st);
}

template <typename T>
static int coarse_solve(Mg *mg, const T *b, T *x, bool tr, hipStream_t st)
{
    FE_CHECK_HIP(mg_coarse_apply<T>((int)mg->nc, (int)mg->nf, mg->Xinv, mg->dmap, mg->dmap + mg->nc, b,
                                    x, mg->cpart, tr, st));
    return FE_OK;
}

template <typename T>
static T *altT(MgLevel &L);
template <>
double *altT<double>(MgLevel &L) { return L.xa; }
template <>
float *altT<float>(MgLevel &L) { return L.xa32; }

// V-cycle from level l on b; x receives the result.  first_done: the first
// pre-smoothing sweep from x = 0 (x = omega D^{-1} b) has already been applied
// to x, by the restriction kernel of the level above (or, at the finest level
// of a mixed-precision cycle, together with the cast of the Krylov vector).
// A damped block-Jacobi sweep x += omega D^{-1} (b - A x) (transposed when tr)
// is fused with the element pass on matrix-free levels, and is one kernel on
// assembled ones, which writes the new iterate to the level's second buffer:
// the iterate alternates between x and that buffer, and ends in x.
template <typename T>
static int vcycle(Mg *mg, int l, const T *b, T *x, bool tr, hipStream_t st, bool first_done = false)
{
    MgLevel &L = mg->lev[l];
    const int nl = (int)mg->lev.size();
    if (l == nl - 1) return coarse_solve<T>(mg, b, x, tr, st);
    const T om = (T)mg->omega;
    const T *D = blocksT<T>(L);
    T *t = vecT<T>(L, 2);
    T *cur = x;
    auto sweep = [&]() -> hipError_t {
        if (L.assembled) {
            T *nxt = cur == x ? altT<T>(L) : x;
            const hipError_t e = mg_stencil_smooth<T>(L.grid.nx, L.grid.ny, L.grid.nz, stencilT<T>(L),
                                                      D, b, cur, nxt, om, tr, st);
            cur = nxt;
            return e;
        }
        return launch_elem_smooth<T>(tr, L.geo, stateT<T>(L), cur, L.gamma, L.s, L.nmask, t,
                                     (T *)L.slots, D, b, om, st);
    };
    if (!first_done) FE_CHECK_HIP(mg_smooth<T>(D, b, nullptr, x, L.nn, om, tr, false, st));
    for (int it = 1; it < mg->nu1; ++it) FE_CHECK_HIP(sweep());
    MgLevel &C = mg->lev[l + 1];
    FE_CHECK_HIP(op<T>(L, cur, t, tr, st));
    T *bc = vecT<T>(C, 0), *xc = vecT<T>(C, 1);
    // below the coarse level's first sweep is fused into the restriction,
    // except where that level is the directly solved coarsest one
    const bool fuse = l + 1 < nl - 1;
    if (fuse)
        FE_CHECK_HIP(mg_restrict_smooth<T>(C.grid, L.grid, b, t, C.nmask, bc, blocksT<T>(C), xc, om,
                                           tr, st));
    else
        FE_CHECK_HIP(mg_restrict<T>(C.grid, L.grid, b, t, C.nmask, bc, st));
    int rc = vcycle<T>(mg, l + 1, bc, xc, tr, st, fuse);
    if (rc) return rc;
    FE_CHECK_HIP(mg_prolong_add<T>(L.grid, C.grid, xc, L.nmask, cur, st));
    for (int it = 0; it < mg->nu2; ++it) FE_CHECK_HIP(sweep());
    if (cur != x) FE_CHECK_HIP(mg_copy<T>(cur, x, L.ndof, st));
    return FE_OK;
}

int mg_apply64(Mg *mg, const double *v, double *z, bool tr, hipStream_t st)
{
    return vcycle<double>(mg, 0, v, z, tr, st);
}

int mg_apply32(Mg *mg, const double *v, float *z, bool tr, hipStream_t st)
{
    MgLevel &L0 = mg->lev[0];
    FE_CHECK_HIP(mg_smooth0_cast(L0.D32, v, L0.b32, z, L0.nn, (float)mg->omega, tr, st));
    return vcycle<float>(mg, 0, L0.b32, z, tr, st, true);
}

}  // namespace fe
