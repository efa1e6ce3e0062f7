// Optimisation loop internals: PDE density filter and MMA state (device side).
#pragma once

#include "fe_internal.h"

namespace fe {

struct FGeo {
    int nx, ny, nz;
    double E[4];  // element matrix entry for corners differing in 0..3 coordinates
};

// Helmholtz filter workspace (fe_filter.hip)
struct Filter {
    FGeo g;
    int64_t nn = 0, ne = 0;
    double load = 0.0;  // h^3 / 8
    double *b = nullptr, *x = nullptr, *r = nullptr, *p = nullptr, *y = nullptr;
    double *partial = nullptr, *sc = nullptr;  // sc: rz[0], rz[1], pAp, rr, rr0
    double *hsc = nullptr;                     // pinned host scalars
    int last_its = 0;
};
hipError_t filter_alloc(Filter *f, const fe_grid &grid, double radius);
void filter_free(Filter *f);
// b = scale * (element-to-node sum of gamma)
hipError_t filter_load(Filter *f, const double *gamma, double scale, hipStream_t st);
// x = K^-1 b by Jacobi-preconditioned CG to relative residual rtol
int filter_solve(Filter *f, hipStream_t st, double rtol, int max_its);
// out = scale * (node-to-element sum of x)
hipError_t filter_unload(Filter *f, double scale, double *out, hipStream_t st);

// MMA state (fe_mma.hip)
struct MmaState {
    int64_t n = 0;
    double xmin = 0, xmax = 1, move = 0.2;
    int k = 0;
    double *xold1 = nullptr, *xold2 = nullptr, *low = nullptr, *upp = nullptr;
    double *al = nullptr, *be = nullptr, *c = nullptr, *partial = nullptr, *sum = nullptr;
    double *hsum = nullptr;
};
hipError_t mma_alloc(MmaState *m);
void mma_free(MmaState *m);
int mma_update(MmaState *m, double *x, const double *df0, double f1, const double *df1,
               double *lam_out, hipStream_t st);

// element-vector helpers (fe_mma.hip)
hipError_t launch_blend(int64_t n, const uint8_t *design, const double *a, const double *b,
                        double *out, hipStream_t st);
hipError_t launch_masked_scale(int64_t n, const uint8_t *design, const double *a, double scale,
                               double *out, hipStream_t st);
hipError_t launch_gather(int64_t nd, const int64_t *idx, const double *full, double *compact,
                         hipStream_t st);
hipError_t launch_scatter(int64_t nd, const int64_t *idx, const double *compact, double *full,
                          hipStream_t st);
// partial[b] = block b's sum over design of (1 - g); partial[RED_BLOCKS + b] = its max |a - b|
hipError_t launch_vol_change(int64_t n, const uint8_t *design, const double *g, int64_t nd,
                             const double *a, const double *b, double *partial, hipStream_t st);

}  // namespace fe
