// Mesh data of the otbb library: the generic two-level FV mesh (Sec. 2.1)
// in ELL form on the device, plus the aggregation hierarchy used by the
// multigrid preconditioner of the per-slice Laplacians.
#pragma once

#include "common.hpp"

namespace otbb {

// One level of the aggregation hierarchy of the fine-cell graph.  The graph
// is the same for every time slice; only the edge weights change per slice.
struct MGLevelHost {
    int n = 0, ne = 0, w = 0;          // cells, edges, ELL width
    std::vector<int> nb, ed;           // [w * n], column-major (t * n + i); -1 pads
    std::vector<int> agg;              // cell -> aggregate at the next level
    std::vector<int> mem_ptr, mem_idx; // next-level aggregate -> member cells
    std::vector<int> cedge_ptr, cedge_idx; // next-level edge -> edges here
};

struct MGLevelDev {
    int n = 0, ne = 0, w = 0, n_next = 0, ne_next = 0;
    DBuf<int> nb, ed, agg, mem_ptr, mem_idx, cedge_ptr, cedge_idx;
};

// One level of the aggregation hierarchy of the coarse (density) cells used
// by the multigrid preconditioner of the pseudo-Schur system.  Level 0 is
// the density cells themselves (operator applied matrix-free); level l >= 1
// holds a Galerkin operator assembled by probing, stored per time offset
// (-1, 0, +1) in ELL form over the level's stencil.
struct SLevelHost {
    int n = 0, w = 0;                  // cells, stencil width (slot 0 = self)
    std::vector<int> nbr;              // [w * n] col-major, -1 pads
    int ncolor = 0;                    // distance-2 coloring over the stencil
    std::vector<int> color;
    std::vector<int> slot_of;          // [ncolor * n]: slot of the colour-c neighbour, -1
    std::vector<int> agg, mem_ptr, mem_idx;   // to the next level (empty at the last)
};

struct SLevelDev {
    int n = 0, w = 0, ncolor = 0, n_next = 0;
    DBuf<int> nbr, color, slot_of, agg, mem_ptr, mem_idx;
};

// Host copy of the description plus every derived index structure.
struct MeshHost {
    int nf = 0, nc = 0, ne = 0, nce = 0;
    int grid_n = 0;                    // > 0: fine cells form a grid_n^grid_dim grid
    int grid_dim = 2;
    std::vector<double> a, ac;
    std::vector<int> ov_f, ov_c;
    std::vector<double> ov_a;
    std::vector<int> eK, eL, erK, erL;
    std::vector<double> elen, edist, elam;
    std::vector<int> ceI, ceJ;
    std::vector<double> celen, cedist, celam;
    // derived
    int wf = 0;                        // fine cell -> edges ELL width
    std::vector<int> cf_edge, cf_nb;   // [wf * nf] col-major, -1 pads
    int wo = 0;                        // fine -> overlapping coarse cells
    std::vector<int> fo_c;
    std::vector<double> fo_w;
    int woc = 0;                       // coarse -> overlapping fine cells
    std::vector<int> co_f;
    std::vector<double> co_w;
    int wr = 0;                        // coarse cell -> fine edge-sides (R_T)
    std::vector<int> cr_e;
    std::vector<double> cr_w;
    int wcc = 0;                       // coarse cell -> coarse edges
    std::vector<int> cc_edge, cc_nb;
    std::vector<MGLevelHost> levels;
    int ncolor = 0;                    // distance coloring of the coarse cells
    std::vector<int> color;            // for probing the pseudo-Schur diagonal
    std::vector<std::vector<int>> cpl; // pseudo-Schur stencil of each coarse cell (no self)
    std::vector<SLevelHost> slevels;   // pseudo-Schur multigrid hierarchy
};

}  // namespace otbb

// The opaque C handle.
struct ot_mesh {
    otbb::MeshHost h;
    int device = 0;
    // device copies (geometry in FP64; kernels convert on load)
    otbb::DBuf<double> a, ac, elam, etw, eW, einvd, elen, cetw, celam, fo_w, co_w, cr_w;
    otbb::DBuf<int> eK, eL, erK, erL, ceI, ceJ, cf_edge, cf_nb, fo_c, co_f, cr_e, cc_edge, cc_nb;
    otbb::DBuf<int> color;
    // R_T stencil of each coarse cell resolved once at setup, same ELL slots
    // as cr_e: the edge's two potential cells and 0.5 cr_w / d_e, so the
    // pseudo-Schur output pass reads them coalesced instead of through the
    // edge index
    otbb::DBuf<int> cr_k, cr_l;
    otbb::DBuf<double> cr_g, cr_g2;
    otbb::DBuf<int> cf_rk, cf_rl;
    otbb::DBuf<double> cf_lam, cf_bw, cf_tw;
    std::vector<otbb::MGLevelDev> lv;
    std::vector<otbb::SLevelDev> slv;
    double area = 0.0;                 // |Omega| = sum of coarse areas
};

namespace otbb {
void mesh_finalize(ot_mesh *m);        // derive structures + upload
void structured_desc(int n, bool cartesian, MeshHost &h);
void cartesian3d_desc(int n, MeshHost &h);
}  // namespace otbb
