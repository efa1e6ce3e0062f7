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
    // small levels: the operator assembled as a 27-point block stencil (675 per node)
    bool assembled = false;
    double *S = nullptr;
    float *S32 = nullptr;
    double *xa = nullptr;   // second iterate buffer of the one-kernel sweeps
    float *xa32 = nullptr;
};

struct Mg {
    fe_problem *owner = nullptr;  // allocations go through owner->alloc
    std::vector<MgLevel> lev;
    bool mixed = false;
    int nu1 = 2, nu2 = 1;  // smoothing sweeps before and after the coarse-grid correction
    double omega = 0.6;
    // coarsest level: band LU on the host of the dense-stored matrix restricted
    // to its nf free DOFs, explicit inverse from its factors on the device
    int64_t nc = 0;          // DOFs of the coarsest level
    int64_t nf = 0;          // of which not prescribed (set per Newton step from the mask)
    int bw = 0;              // half bandwidth of the full coarsest matrix (buffer sizing)
    int kl = 0, ku = 0;      // half bandwidths of the condensed matrix (<= bw)
    std::vector<double> A;   // dense work matrix of the factorisation, nf x nf
    double *hfac = nullptr;  // pinned: L by columns [nf kl], U above the diagonal by columns
                             // [nf (kl + ku)], diagonal of U [nf]
    int *hpiv = nullptr;     // pinned: pivot rows [nf]
    uint8_t *hmask = nullptr;  // pinned: node mask of the coarsest level
    int *hmap = nullptr;     // pinned: free -> full DOF index [nc] (first nf used), then
                             // full -> free index or -1 for a prescribed DOF [nc]
    double *dfac = nullptr;  // device copy of hfac
    int *dpiv = nullptr;     // device copy of hpiv
    int *dmap = nullptr;     // device copy of hmap
    double *Xinv = nullptr;  // device: inverse of the condensed matrix by columns, nf x nf
    double *cpart = nullptr; // device: row partials of the coarse product, ceil(nf / 64) x nf
    hipEvent_t probe_ready = nullptr;  // the probing products have reached the host
    int64_t asm_nodes = 0;        // levels with at most this many nodes are assembled
    double *probe = nullptr;      // element Jacobians (coarsest or assembled level), 1600 per element
    double *probe_out = nullptr;  // 135 probing products, [q][n_dof]
    double *hbuf = nullptr;
    // The coarsest level's factorisation (Xinv, index maps) can be kept from
    // one Newton step to the next: reuse_coarse is set by the caller for a
    // set-up; coarse_ready says a factorisation of the current design exists.
    bool reuse_coarse = false, coarse_ready = false, skip_coarse = false;
};

// Dense row-major n_dof x n_dof J of a grid from its 135 probing products
// (probe: [q][n_dof] on the host).
void assemble_from_probes(const fe_grid &grid, const double *probe, double *A);

// Default node-count limit of assembled levels (an assembled level streams 675
// stencil entries per node instead of running the element pass, whose latency
// does not shrink with the grid).
constexpr int64_t MG_ASM_NODES_DEFAULT = 10000;
int64_t mg_asm_nodes(int opt);  // option value -> limit (-1: default, 0: none)

int mg_num_levels(const fe_grid &g);
int64_t mg_footprint_bytes(const fe_grid &g, bool mixed, int64_t asm_nodes);
int mg_create(fe_problem *p, bool mixed, int64_t asm_nodes, Mg **out);
void mg_free(Mg *mg);
int mg_set_design(Mg *mg, fe_problem *p, const double *gamma, const double *s, hipStream_t st);
// Per Newton step: mg_setup_begin before the caller's fine-level block diagonal
// (it starts the coarsest level's probing products), mg_setup_finish after it.
// D0 / D032, x032: the finest level's inverted blocks and FP32 state.  A
// mixed-precision step passes D032 and x032 (its V-cycles run in FP32, and the
// blocks of the other matrix-free levels are then formed in FP32 only); an FP64
// step (or the adjoint) passes NULL for both and gets FP64 blocks.
int mg_setup_begin(Mg *mg, fe_problem *p, const double *x, hipStream_t st);
int mg_setup_finish(Mg *mg, fe_problem *p, const double *D0, const float *D032, const float *x032,
                    hipStream_t st);
// z = M v with M one V-cycle (for J, or for J^T when tr)
int mg_apply64(Mg *mg, const double *v, double *z, bool tr, hipStream_t st);
int mg_apply32(Mg *mg, const double *v, float *z, bool tr, hipStream_t st);

}  // namespace fe
