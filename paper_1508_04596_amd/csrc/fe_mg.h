// Geometric multigrid preconditioner: hierarchy and entry points (internal).
#pragma once

#include <vector>

#include "fe_internal.h"

namespace fe {

struct MgLevel {
    fe_grid grid;
    Geo geo;
    int64_t nn = 0, ne = 0, ndof = 0;
    uint8_t *nmask = nullptr;              // per-node prescribed bits
    double *gamma = nullptr, *s = nullptr; // element design and source
    double *x = nullptr;                   // linearisation state
    float *x32 = nullptr;
    double *D = nullptr;                   // inverted nodal blocks
    float *D32 = nullptr;
    double *slots = nullptr, *slots25 = nullptr;
    double *b = nullptr, *xs = nullptr, *t = nullptr;    // FP64 rhs, correction, work
    float *b32 = nullptr, *xs32 = nullptr, *t32 = nullptr;
};

struct Mg {
    fe_problem *owner = nullptr;  // allocations go through owner->alloc
    std::vector<MgLevel> lev;
    bool mixed = false;
    int nu1 = 2, nu2 = 2;
    double omega = 0.6;
    // coarsest level: dense-stored band LU
    int64_t nc = 0;
    int kl = 0, ku = 0;
    std::vector<double> A, hb, Lc;  // dense band LU, work vector, L multipliers by column
    std::vector<double> Uc;         // U by columns, kl + ku entries above the diagonal each
    std::vector<int> piv;
    double *probe = nullptr;      // element Jacobians of the coarsest level, 1600 per element
    double *probe_out = nullptr;  // 135 probing products, [q][n_dof]
    double *hbuf = nullptr;
};

// Dense row-major n_dof x n_dof J of a grid from its 135 probing products
// (probe: [q][n_dof] on the host).
void assemble_from_probes(const fe_grid &grid, const double *probe, double *A);

int mg_num_levels(const fe_grid &g);
int64_t mg_footprint_bytes(const fe_grid &g, bool mixed);
int mg_create(fe_problem *p, bool mixed, Mg **out);
void mg_free(Mg *mg);
int mg_set_design(Mg *mg, fe_problem *p, const double *gamma, const double *s, hipStream_t st);
int mg_setup(Mg *mg, fe_problem *p, const double *x, const double *D0, const float *D032,
             const float *x032, hipStream_t st);
// z = M v with M one V-cycle (for J, or for J^T when tr)
int mg_apply64(Mg *mg, const double *v, double *z, bool tr, hipStream_t st);
int mg_apply32(Mg *mg, const double *v, float *z, bool tr, hipStream_t st);

}  // namespace fe
