// Internal interface of the block-local deflation (dfl.hip) used by GCR.
#pragma once
#include "internal.h"

struct qcd_dfl_s {
    qcd_field f = nullptr;
    int device = 0;
    qcd_dfl_params params{};
    int Ns = 0, Nb = 0;        // Nb: deflation blocks
    int r = 1;                 // Schwarz blocks per deflation block
    dfl::Geom dg{};            // deflation-block geometry (b = deflation block, nb its grid)
    // Phi: [Nb][Ns][r members][6 chunks][2 parities][Vbh] float4: deflation
    // blocks in lexicographic order of their grid, member Schwarz blocks in
    // lexicographic order inside, sites of a member in the internal (parity, j) order
    float4 *phi = nullptr;
    double2 *A = nullptr;      // little operator [Nb][9][Ns][Ns], d = 0 self, 1+2mu+dir neighbours
    double2 *Dinv = nullptr;   // inverse diagonal blocks [Nb][Ns][Ns]
    int *bnbr = nullptr;       // [Nb][9] neighbour deflation block (lexicographic), d as for A
    int *brow = nullptr;       // [Nb] deflation blocks by colour: the Nb/2 even ones, then the odd ones
    int *boff = nullptr;       // [Nb][r] internal site offset (rank * Vbh) of each member Schwarz block
    int *dbof = nullptr;       // [Schwarz blocks] deflation block of the Schwarz block of memory rank k
    int *loc = nullptr;        // [V] internal site -> lexicographic site index inside its deflation block
    int *blex = nullptr;       // [V] internal site -> lexicographic deflation block index
    // grow-only work space for little-vector algebra
    void *lw = nullptr;
    size_t lw_bytes = 0;
    double *hp = nullptr;      // pinned host scratch
};

namespace dfl {

qcd_field dfl_field(qcd_dfl d);
// x += Phi A^{-1} Phi^+ b for FP64 internal vectors; the little system is
// solved to relative residual tol (at most maxit iterations)
// x += Phi A^{-1} Phi^+ b (set: x = ...)
int dfl_low_mode(qcd_dfl d, const double2 *b, double2 *x, int n, double tol, int maxit, bool set, hipStream_t s);
// z <- P_R z = z - Phi A^{-1} Phi^+ M z, vectors of precision vec (F32 or F64); tmp is n vectors of
// scratch; the little system gets a fixed budget of maxit iterations (no host synchronisation)
int dfl_project_R(qcd_dfl d, void *z, void *tmp, int n, qcd_prec vec, qcd_prec storage, int maxit,
                  hipStream_t s);

}  // namespace dfl
