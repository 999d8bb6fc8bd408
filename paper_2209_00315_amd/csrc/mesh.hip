// Mesh construction, validation and derived index structures (host side).
//
// The generic description follows Sec. 2.1: fine cells carry the potential,
// coarse cells carry the density; Omega = M J holds the overlap areas; every
// interior fine edge knows its two cells, the coarse cells feeding the
// density reconstruction on each side, its length, the distance between the
// cell centres and the reconstruction weight lambda.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <set>
#include <unordered_map>

#include "mesh.hpp"

namespace otbb {

// ---------------------------------------------------------------------------
// Structured meshes
// ---------------------------------------------------------------------------
// n x n right-triangle grid.  The two triangles of a fine square share their
// circumcentre (hypotenuse midpoint), so the two-point flux distance across
// the square's diagonal vanishes and the potential is one value per square:
// phi-cells are the n^2 squares (index b*n + a).  Density cells are the
// triangles of the (n/2)^2 coarse squares of side H = 2h, split along the
// SW-NE diagonal: index 2*(B*(n/2) + A) + t, t = 0 for the lower-right
// triangle (x >= y inside the square), t = 1 for the upper-left one.
// Each fine triangle lies in exactly one coarse triangle; the overlap of a
// fine square with a coarse triangle is h^2 or h^2/2.
// Fine edges: interior axis-aligned sides, length = distance = h, lambda 1/2.
// Coarse edges: legs (length = distance = H) and the coarse diagonals, where
// the circumcentre distance vanishes again and the centroid distance
// sqrt(2) H / 3 is used; they only enter the BB coarse Laplacian.
static inline int cidx(int n, int A, int B, int t) { return 2 * (B * (n / 2) + A) + t; }

// coarse triangle holding the lower-right (lr = true) or upper-left half of
// fine square (a, b)
static int parent_of(int n, int a, int b, bool lr) {
    int A = a / 2, B = b / 2, la = a & 1, lb = b & 1;
    if (la == 1 && lb == 0) return cidx(n, A, B, 0);      // square below the coarse diagonal
    if (la == 0 && lb == 1) return cidx(n, A, B, 1);      // square above it
    return cidx(n, A, B, lr ? 0 : 1);                     // diagonal squares: halves split
}

void structured_desc(int n, bool cartesian, MeshHost &h) {
    OT_REQUIRE(n >= 2, OT_EINVAL, "structured mesh: n must be >= 2");
    h = MeshHost();
    const double hh = 1.0 / n;
    h.grid_n = n;
    h.nf = n * n;
    auto add_fine_edges = [&](auto rho_side) {
        for (int b = 0; b < n; ++b)
            for (int a = 0; a + 1 < n; ++a) {          // vertical side x = (a+1) h
                int K = b * n + a, L = b * n + a + 1;
                h.eK.push_back(K); h.eL.push_back(L);
                h.erK.push_back(rho_side(a, b, true, 0));
                h.erL.push_back(rho_side(a + 1, b, false, 0));
            }
        for (int b = 0; b + 1 < n; ++b)
            for (int a = 0; a < n; ++a) {              // horizontal side y = (b+1) h
                int K = b * n + a, L = (b + 1) * n + a;
                h.eK.push_back(K); h.eL.push_back(L);
                h.erK.push_back(rho_side(a, b, false, 1));
                h.erL.push_back(rho_side(a, b + 1, true, 1));
            }
        h.ne = (int)h.eK.size();
        h.elen.assign(h.ne, hh);
        h.edist.assign(h.ne, hh);
        h.elam.assign(h.ne, 0.5);
    };
    if (cartesian) {
        h.nc = n * n;
        h.a.assign(h.nf, hh * hh);
        h.ac.assign(h.nc, hh * hh);
        for (int i = 0; i < h.nf; ++i) { h.ov_f.push_back(i); h.ov_c.push_back(i); h.ov_a.push_back(hh * hh); }
        add_fine_edges([&](int a, int b, bool, int) { return b * n + a; });
        h.ceI = h.eK; h.ceJ = h.eL;
        h.celen = h.elen; h.cedist = h.edist; h.celam = h.elam;
        h.nce = h.ne;
        return;
    }
    OT_REQUIRE(n >= 2 && n % 2 == 0, OT_EINVAL, "structured mesh: n must be even and >= 2");
    const int m = n / 2;
    const double H = 2.0 * hh;
    h.nc = 2 * m * m;
    h.a.assign(h.nf, hh * hh);
    h.ac.assign(h.nc, 2.0 * hh * hh);
    for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
            int i = b * n + a;
            int pl = parent_of(n, a, b, true), pu = parent_of(n, a, b, false);
            if (pl == pu) {
                h.ov_f.push_back(i); h.ov_c.push_back(pl); h.ov_a.push_back(hh * hh);
            } else {
                h.ov_f.push_back(i); h.ov_c.push_back(pl); h.ov_a.push_back(0.5 * hh * hh);
                h.ov_f.push_back(i); h.ov_c.push_back(pu); h.ov_a.push_back(0.5 * hh * hh);
            }
        }
    // The side of square (a, b) on its right or bottom border belongs to its
    // lower-right triangle; the left or top border to its upper-left one.
    add_fine_edges([&](int a, int b, bool right_or_bottom, int) {
        return parent_of(n, a, b, right_or_bottom);
    });
    for (int B = 0; B < m; ++B)
        for (int A = 0; A < m; ++A) {
            h.ceI.push_back(cidx(n, A, B, 0)); h.ceJ.push_back(cidx(n, A, B, 1));
            h.celen.push_back(std::sqrt(2.0) * H); h.cedist.push_back(std::sqrt(2.0) * H / 3.0);
        }
    for (int B = 0; B < m; ++B)
        for (int A = 0; A + 1 < m; ++A) {
            h.ceI.push_back(cidx(n, A, B, 0)); h.ceJ.push_back(cidx(n, A + 1, B, 1));
            h.celen.push_back(H); h.cedist.push_back(H);
        }
    for (int B = 0; B + 1 < m; ++B)
        for (int A = 0; A < m; ++A) {
            h.ceI.push_back(cidx(n, A, B, 1)); h.ceJ.push_back(cidx(n, A, B + 1, 0));
            h.celen.push_back(H); h.cedist.push_back(H);
        }
    h.nce = (int)h.ceI.size();
    h.celam.assign(h.nce, 0.5);
}

// The n x n x n grid of cubes on [0,1]^3 for both levels (J = identity): the
// three-dimensional workload of Sec. 4.1.  Cell (c n + b) n + a; the TPFA
// edges are the interior faces, |e| = h^2, d_e = h, lambda_e = 1/2, with K
// the cell of smaller coordinate along the normal; volumes h^3.  The coarse
// edges of the BB coarse Laplacian are the same faces.
void cartesian3d_desc(int n, MeshHost &h) {
    OT_REQUIRE(n >= 2 && n <= 1024, OT_EINVAL, "3-D Cartesian mesh: n must be in [2, 1024]");
    h = MeshHost();
    const double hh = 1.0 / n, vol = hh * hh * hh;
    h.grid_n = n;
    h.grid_dim = 3;
    h.nf = h.nc = n * n * n;
    h.a.assign(h.nf, vol);
    h.ac.assign(h.nc, vol);
    for (int i = 0; i < h.nf; ++i) { h.ov_f.push_back(i); h.ov_c.push_back(i); h.ov_a.push_back(vol); }
    auto id = [n](int a, int b, int c) { return (c * n + b) * n + a; };
    for (int c = 0; c < n; ++c)
        for (int b = 0; b < n; ++b)
            for (int a = 0; a + 1 < n; ++a) { h.eK.push_back(id(a, b, c)); h.eL.push_back(id(a + 1, b, c)); }
    for (int c = 0; c < n; ++c)
        for (int b = 0; b + 1 < n; ++b)
            for (int a = 0; a < n; ++a) { h.eK.push_back(id(a, b, c)); h.eL.push_back(id(a, b + 1, c)); }
    for (int c = 0; c + 1 < n; ++c)
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) { h.eK.push_back(id(a, b, c)); h.eL.push_back(id(a, b, c + 1)); }
    h.ne = (int)h.eK.size();
    h.erK = h.eK;
    h.erL = h.eL;
    h.elen.assign(h.ne, hh * hh);
    h.edist.assign(h.ne, hh);
    h.elam.assign(h.ne, 0.5);
    h.ceI = h.eK; h.ceJ = h.eL;
    h.celen = h.elen; h.cedist = h.edist; h.celam = h.elam;
    h.nce = h.ne;
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
static void validate(const MeshHost &h) {
    OT_REQUIRE(h.nf > 0 && h.nc > 0, OT_EINVAL, "mesh: empty cell sets");
    OT_REQUIRE(h.ne >= 0 && h.nce >= 0, OT_EINVAL, "mesh: negative edge count");
    for (double x : h.a) OT_REQUIRE(std::isfinite(x) && x > 0, OT_EMESH, "mesh: fine area <= 0");
    for (double x : h.ac) OT_REQUIRE(std::isfinite(x) && x > 0, OT_EMESH, "mesh: coarse area <= 0");
    std::vector<double> rs(h.nf, 0.0), cs(h.nc, 0.0);
    for (size_t t = 0; t < h.ov_f.size(); ++t) {
        OT_REQUIRE(h.ov_f[t] >= 0 && h.ov_f[t] < h.nf && h.ov_c[t] >= 0 && h.ov_c[t] < h.nc,
                   OT_EMESH, "mesh: overlap index out of range");
        OT_REQUIRE(std::isfinite(h.ov_a[t]) && h.ov_a[t] >= 0, OT_EMESH, "mesh: negative overlap");
        rs[h.ov_f[t]] += h.ov_a[t];
        cs[h.ov_c[t]] += h.ov_a[t];
    }
    for (int i = 0; i < h.nf; ++i)
        OT_REQUIRE(std::fabs(rs[i] - h.a[i]) <= 1e-10 * h.a[i], OT_EMESH,
                   "mesh: overlaps of a fine cell do not sum to its area");
    for (int j = 0; j < h.nc; ++j)
        OT_REQUIRE(std::fabs(cs[j] - h.ac[j]) <= 1e-10 * h.ac[j], OT_EMESH,
                   "mesh: overlaps of a coarse cell do not sum to its area");
    for (int e = 0; e < h.ne; ++e) {
        OT_REQUIRE(h.eK[e] >= 0 && h.eK[e] < h.nf && h.eL[e] >= 0 && h.eL[e] < h.nf && h.eK[e] != h.eL[e],
                   OT_EMESH, "mesh: bad fine edge cells");
        OT_REQUIRE(h.erK[e] >= 0 && h.erK[e] < h.nc && h.erL[e] >= 0 && h.erL[e] < h.nc,
                   OT_EMESH, "mesh: bad density side of a fine edge");
        OT_REQUIRE(std::isfinite(h.elen[e]) && h.elen[e] > 0 && std::isfinite(h.edist[e]) && h.edist[e] > 0,
                   OT_EMESH, "mesh: fine edge length or distance <= 0");
        OT_REQUIRE(h.elam[e] >= 0 && h.elam[e] <= 1, OT_EMESH, "mesh: lambda outside [0,1]");
    }
    for (int e = 0; e < h.nce; ++e) {
        OT_REQUIRE(h.ceI[e] >= 0 && h.ceI[e] < h.nc && h.ceJ[e] >= 0 && h.ceJ[e] < h.nc && h.ceI[e] != h.ceJ[e],
                   OT_EMESH, "mesh: bad coarse edge cells");
        OT_REQUIRE(std::isfinite(h.celen[e]) && h.celen[e] > 0 && std::isfinite(h.cedist[e]) && h.cedist[e] > 0,
                   OT_EMESH, "mesh: coarse edge length or distance <= 0");
        OT_REQUIRE(h.celam[e] >= 0 && h.celam[e] <= 1, OT_EMESH, "mesh: coarse lambda outside [0,1]");
    }
}

// ---------------------------------------------------------------------------
// Derived ELL structures
// ---------------------------------------------------------------------------
// Pack ragged lists into a column-major ELL array (t * n + i), padding -1.
template <typename T>
static int pack_ell(const std::vector<std::vector<std::pair<int, T>>> &rows,
                    std::vector<int> &idx, std::vector<T> &val) {
    int n = (int)rows.size(), w = 0;
    for (auto &r : rows) w = std::max(w, (int)r.size());
    w = std::max(w, 1);
    idx.assign((size_t)w * n, -1);
    val.assign((size_t)w * n, T(0));
    for (int i = 0; i < n; ++i)
        for (size_t t = 0; t < rows[i].size(); ++t) {
            idx[t * n + i] = rows[i][t].first;
            val[t * n + i] = rows[i][t].second;
        }
    return w;
}

// Aggregation of a graph (cells + edges) into the next multigrid level.
// Grid graphs (fine cells of the structured meshes) use 2 x 2 blocks; other
// graphs a greedy root-plus-neighbours aggregation followed by attaching
// leftovers to the neighbouring aggregate they share most edges with.
static void aggregate(int n, int gridn, const std::vector<int> &ei, const std::vector<int> &ej,
                      std::vector<int> &agg, int &nagg, int griddim = 2) {
    agg.assign(n, -1);
    if (gridn > 0 && griddim == 3) {
        int g2 = (gridn + 1) / 2;
        for (int i = 0; i < n; ++i) {
            int c = i / (gridn * gridn), r = i % (gridn * gridn), b = r / gridn, a = r % gridn;
            agg[i] = ((c / 2) * g2 + b / 2) * g2 + a / 2;
        }
        nagg = g2 * g2 * g2;
        return;
    }
    if (gridn > 0) {
        int g2 = (gridn + 1) / 2;
        for (int i = 0; i < n; ++i) {
            int b = i / gridn, a = i % gridn;
            agg[i] = (b / 2) * g2 + a / 2;
        }
        nagg = g2 * g2;
        return;
    }
    std::vector<std::vector<int>> adj(n);
    for (size_t e = 0; e < ei.size(); ++e) { adj[ei[e]].push_back(ej[e]); adj[ej[e]].push_back(ei[e]); }
    nagg = 0;
    for (int i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        bool free_nb = true;
        for (int j : adj[i]) if (agg[j] >= 0) { free_nb = false; break; }
        if (!free_nb) continue;
        agg[i] = nagg;
        for (int j : adj[i]) agg[j] = nagg;
        ++nagg;
    }
    for (int i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        std::map<int, int> cnt;
        for (int j : adj[i]) if (agg[j] >= 0) cnt[agg[j]]++;
        int best = -1, bc = 0;
        for (auto &kv : cnt) if (kv.second > bc) { bc = kv.second; best = kv.first; }
        if (best >= 0) agg[i] = best;
    }
    for (int i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        agg[i] = nagg;
        for (int j : adj[i]) if (agg[j] < 0) agg[j] = nagg;
        ++nagg;
    }
}

static void build_hierarchy(MeshHost &h) {
    h.levels.clear();
    std::vector<int> ei = h.eK, ej = h.eL;
    int n = h.nf, gridn = h.grid_n;
    for (int lvl = 0; lvl < 24; ++lvl) {
        MGLevelHost L;
        L.n = n;
        L.ne = (int)ei.size();
        // (edge, neighbour): the edge column is padded with -1, which the
        // kernels use to stop; the neighbour column pads with a valid 0
        std::vector<std::vector<std::pair<int, int>>> rows(n);
        for (int e = 0; e < L.ne; ++e) {
            rows[ei[e]].push_back({e, ej[e]});
            rows[ej[e]].push_back({e, ei[e]});
        }
        L.w = pack_ell(rows, L.ed, L.nb);
        bool last = n <= 4 || L.ne == 0;
        if (!last) {
            int nagg = 0;
            aggregate(n, gridn, ei, ej, L.agg, nagg, h.grid_dim);
            if (nagg >= n) last = true;
            else {
                // members of each aggregate
                L.mem_ptr.assign(nagg + 1, 0);
                for (int i = 0; i < n; ++i) L.mem_ptr[L.agg[i] + 1]++;
                for (int c = 0; c < nagg; ++c) L.mem_ptr[c + 1] += L.mem_ptr[c];
                L.mem_idx.assign(n, 0);
                std::vector<int> pos(L.mem_ptr.begin(), L.mem_ptr.end() - 1);
                for (int i = 0; i < n; ++i) L.mem_idx[pos[L.agg[i]]++] = i;
                // coarse edges: pairs of distinct aggregates joined by an edge
                std::map<std::pair<int, int>, int> key;
                std::vector<int> nei, nej, emap(L.ne, -1);
                for (int e = 0; e < L.ne; ++e) {
                    int u = L.agg[ei[e]], v = L.agg[ej[e]];
                    if (u == v) continue;
                    auto k = std::make_pair(std::min(u, v), std::max(u, v));
                    auto it = key.find(k);
                    if (it == key.end()) {
                        it = key.emplace(k, (int)nei.size()).first;
                        nei.push_back(k.first);
                        nej.push_back(k.second);
                    }
                    emap[e] = it->second;
                }
                int nce = (int)nei.size();
                L.cedge_ptr.assign(nce + 1, 0);
                for (int e = 0; e < L.ne; ++e) if (emap[e] >= 0) L.cedge_ptr[emap[e] + 1]++;
                for (int c = 0; c < nce; ++c) L.cedge_ptr[c + 1] += L.cedge_ptr[c];
                L.cedge_idx.assign(L.cedge_ptr[nce], 0);
                std::vector<int> p2(L.cedge_ptr.begin(), L.cedge_ptr.end() - 1);
                for (int e = 0; e < L.ne; ++e) if (emap[e] >= 0) L.cedge_idx[p2[emap[e]]++] = e;
                ei = nei; ej = nej;
                n = nagg;
                gridn = gridn > 0 ? (gridn + 1) / 2 : 0;
            }
        }
        h.levels.push_back(std::move(L));
        if (last) break;
    }
    // the last level carries no aggregation data
    h.levels.back().agg.clear();
    h.levels.back().mem_ptr.clear();
    h.levels.back().mem_idx.clear();
    h.levels.back().cedge_ptr.clear();
    h.levels.back().cedge_idx.clear();
}

// Greedy coloring of the coarse cells such that two cells of one color are
// never coupled by the pseudo-Schur operator of the BB preconditioner (its
// stencil: coarse edges, plus coarse cells reached through the fine cells
// within one fine edge of the overlap of a coarse cell).  Probing with one
// color at a time then returns exact diagonal entries.
static void color_coarse(MeshHost &h) {
    std::vector<std::vector<int>> f_of_c(h.nc), c_of_f(h.nf), fadj(h.nf);
    for (size_t t = 0; t < h.ov_f.size(); ++t) {
        if (h.ov_a[t] == 0) continue;
        f_of_c[h.ov_c[t]].push_back(h.ov_f[t]);
        c_of_f[h.ov_f[t]].push_back(h.ov_c[t]);
    }
    for (int e = 0; e < h.ne; ++e) {
        fadj[h.eK[e]].push_back(h.eL[e]);
        fadj[h.eL[e]].push_back(h.eK[e]);
        for (int c : {h.erK[e], h.erL[e]}) { c_of_f[h.eK[e]].push_back(c); c_of_f[h.eL[e]].push_back(c); }
    }
    std::vector<std::set<int>> cpl(h.nc);
    for (int j = 0; j < h.nc; ++j) {
        std::set<int> F;
        for (int i : f_of_c[j]) { F.insert(i); for (int q : fadj[i]) F.insert(q); }
        for (int i : F) for (int c : c_of_f[i]) if (c != j) cpl[j].insert(c);
    }
    for (int e = 0; e < h.nce; ++e) { cpl[h.ceI[e]].insert(h.ceJ[e]); cpl[h.ceJ[e]].insert(h.ceI[e]); }
    for (int j = 0; j < h.nc; ++j)
        for (int c : cpl[j]) cpl[c].insert(j);        // symmetric closure
    h.cpl.assign(h.nc, {});
    for (int j = 0; j < h.nc; ++j) h.cpl[j].assign(cpl[j].begin(), cpl[j].end());
    h.color.assign(h.nc, -1);
    h.ncolor = 0;
    std::vector<int> mark;
    for (int j = 0; j < h.nc; ++j) {
        mark.assign(h.ncolor + 1, 0);
        for (int c : cpl[j]) if (h.color[c] >= 0) mark[h.color[c]] = 1;
        int col = 0;
        while (mark[col]) ++col;
        h.color[j] = col;
        h.ncolor = std::max(h.ncolor, col + 1);
    }
}

// Pseudo-Schur multigrid hierarchy over the density cells.  Aggregation
// follows the coarse edge graph (root plus neighbours, then leftovers join
// the aggregate they touch most); the stencil of level l+1 is the union of
// the stencils of the member cells; a distance-2 coloring of every coarse
// level lets one probe per (time class, colour) recover its Galerkin
// operator exactly.
static void build_schur_hierarchy(MeshHost &h) {
    h.slevels.clear();
    std::vector<std::vector<int>> st(h.nc);
    for (int j = 0; j < h.nc; ++j) {
        st[j].push_back(j);
        for (int c : h.cpl[j]) st[j].push_back(c);
    }
    std::vector<int> ei = h.ceI, ej = h.ceJ;
    int n = h.nc;
    for (int lvl = 0; lvl < 16; ++lvl) {
        SLevelHost L;
        L.n = n;
        L.w = 1;
        for (auto &r : st) L.w = std::max(L.w, (int)r.size());
        L.nbr.assign((size_t)L.w * n, -1);
        for (int a = 0; a < n; ++a)
            for (size_t t = 0; t < st[a].size(); ++t) L.nbr[t * n + a] = st[a][t];
        if (lvl > 0) {
            // distance-2 coloring: the columns of every row get distinct colours
            L.color.assign(n, -1);
            std::vector<int> mark;
            for (int b = 0; b < n; ++b) {
                mark.assign(L.ncolor + 1, 0);
                for (int a : st[b])
                    for (int c : st[a])
                        if (L.color[c] >= 0 && L.color[c] <= L.ncolor) mark[L.color[c]] = 1;
                int col = 0;
                while (col < (int)mark.size() && mark[col]) ++col;
                L.color[b] = col;
                L.ncolor = std::max(L.ncolor, col + 1);
            }
            L.slot_of.assign((size_t)L.ncolor * n, -1);
            for (int a = 0; a < n; ++a)
                for (size_t t = 0; t < st[a].size(); ++t) {
                    int &slot = L.slot_of[(size_t)L.color[st[a][t]] * n + a];
                    OT_REQUIRE(slot < 0, OT_EMESH, "internal: coloring not distance-2");
                    slot = (int)t;
                }
        }
        bool last = n <= 16;
        std::vector<int> agg;
        int nagg = 0;
        if (!last) {
            aggregate(n, 0, ei, ej, agg, nagg);
            if (nagg > (9 * n) / 10 || nagg < 1) last = true;
        }
        if (!last) {
            L.agg = agg;
            L.mem_ptr.assign(nagg + 1, 0);
            for (int i = 0; i < n; ++i) L.mem_ptr[agg[i] + 1]++;
            for (int c = 0; c < nagg; ++c) L.mem_ptr[c + 1] += L.mem_ptr[c];
            L.mem_idx.assign(n, 0);
            std::vector<int> pos(L.mem_ptr.begin(), L.mem_ptr.end() - 1);
            for (int i = 0; i < n; ++i) L.mem_idx[pos[agg[i]]++] = i;
            // next stencil and aggregation graph
            std::vector<std::set<int>> ns(nagg);
            for (int a = 0; a < n; ++a)
                for (int b : st[a]) ns[agg[a]].insert(agg[b]);
            std::set<std::pair<int, int>> ne;
            for (size_t e = 0; e < ei.size(); ++e) {
                int u = agg[ei[e]], v = agg[ej[e]];
                if (u != v) ne.insert({std::min(u, v), std::max(u, v)});
            }
            std::vector<std::vector<int>> nst(nagg);
            for (int a = 0; a < nagg; ++a) {
                nst[a].push_back(a);
                for (int b : ns[a]) if (b != a) nst[a].push_back(b);
            }
            st.swap(nst);
            ei.clear(); ej.clear();
            for (auto &pr : ne) { ei.push_back(pr.first); ej.push_back(pr.second); }
            n = nagg;
        }
        h.slevels.push_back(std::move(L));
        if (last) break;
    }
}

static void derive(MeshHost &h) {
    {   // fine cell -> (edge, neighbour)
        std::vector<std::vector<std::pair<int, int>>> rows(h.nf);
        for (int e = 0; e < h.ne; ++e) {
            rows[h.eK[e]].push_back({e, h.eL[e]});
            rows[h.eL[e]].push_back({e, h.eK[e]});
        }
        h.wf = pack_ell(rows, h.cf_edge, h.cf_nb);
    }
    {   // Omega by rows and by columns
        std::vector<std::vector<std::pair<int, double>>> fr(h.nf), cr(h.nc);
        for (size_t t = 0; t < h.ov_f.size(); ++t) {
            fr[h.ov_f[t]].push_back({h.ov_c[t], h.ov_a[t]});
            cr[h.ov_c[t]].push_back({h.ov_f[t], h.ov_a[t]});
        }
        h.wo = pack_ell(fr, h.fo_c, h.fo_w);
        h.woc = pack_ell(cr, h.co_f, h.co_w);
    }
    {   // R_T = R_E^T W: coarse cell j gathers lambda W from edges whose K
        // side density is j and (1 - lambda) W from edges whose L side is j
        std::vector<std::map<int, double>> acc(h.nc);
        for (int e = 0; e < h.ne; ++e) {
            double W = h.elen[e] * h.edist[e];
            acc[h.erK[e]][e] += h.elam[e] * W;
            acc[h.erL[e]][e] += (1.0 - h.elam[e]) * W;
        }
        std::vector<std::vector<std::pair<int, double>>> rows(h.nc);
        for (int j = 0; j < h.nc; ++j)
            for (auto &kv : acc[j]) rows[j].push_back(kv);
        h.wr = pack_ell(rows, h.cr_e, h.cr_w);
    }
    {   // coarse cell -> (coarse edge, neighbour)
        std::vector<std::vector<std::pair<int, int>>> rows(h.nc);
        for (int e = 0; e < h.nce; ++e) {
            rows[h.ceI[e]].push_back({e, h.ceJ[e]});
            rows[h.ceJ[e]].push_back({e, h.ceI[e]});
        }
        h.wcc = pack_ell(rows, h.cc_edge, h.cc_nb);
    }
    build_hierarchy(h);
    color_coarse(h);
    build_schur_hierarchy(h);
    // Every kernel walks an ELL row until its stop column reads -1 and then
    // gathers through the paired column: check that padding is contiguous
    // and every gathered index is in range before anything reaches a device.
    auto ell_ok = [](const std::vector<int> &stop, const std::vector<int> &gather, int w, int n, int nstop,
                     int ngather) {
        for (int i = 0; i < n; ++i) {
            bool ended = false;
            for (int t = 0; t < w; ++t) {
                int sidx = stop[(size_t)t * n + i];
                if (sidx < 0) { ended = true; continue; }
                if (ended || sidx >= nstop) return false;
                if (!gather.empty()) {
                    int g = gather[(size_t)t * n + i];
                    if (g < 0 || g >= ngather) return false;
                }
            }
        }
        return true;
    };
    bool ok = ell_ok(h.cf_edge, h.cf_nb, h.wf, h.nf, h.ne, h.nf) &&
              ell_ok(h.fo_c, {}, h.wo, h.nf, h.nc, 0) && ell_ok(h.co_f, {}, h.woc, h.nc, h.nf, 0) &&
              ell_ok(h.cr_e, {}, h.wr, h.nc, h.ne, 0) && ell_ok(h.cc_edge, h.cc_nb, h.wcc, h.nc, h.nce, h.nc);
    for (const MGLevelHost &L : h.levels) ok = ok && ell_ok(L.ed, L.nb, L.w, L.n, std::max(L.ne, 1), L.n);
    for (size_t l = 0; l < h.slevels.size(); ++l) {
        const SLevelHost &L = h.slevels[l];
        ok = ok && ell_ok(L.nbr, {}, L.w, L.n, L.n, 0);
        for (int a = 0; a < L.n; ++a) ok = ok && L.nbr[a] == a;             // slot 0 is the cell itself
        if (!L.agg.empty()) {
            const int nn = (int)L.mem_ptr.size() - 1;
            for (int a : L.agg) ok = ok && a >= 0 && a < nn;
            ok = ok && l + 1 < h.slevels.size() && h.slevels[l + 1].n == nn;
        }
    }
    OT_REQUIRE(ok, OT_EMESH, "internal: inconsistent ELL index structure");
}

void derive_host_only(MeshHost &h) {
    validate(h);
    derive(h);
}

void mesh_finalize(ot_mesh *m) {
    MeshHost &h = m->h;
    validate(h);
    derive(h);
    OT_HIP(hipGetDevice(&m->device));
    hipStream_t s = nullptr;
    m->area = std::accumulate(h.ac.begin(), h.ac.end(), 0.0);
    std::vector<double> tw(h.ne), W(h.ne), invd(h.ne), ctw(h.nce);
    for (int e = 0; e < h.ne; ++e) {
        tw[e] = h.elen[e] / h.edist[e];
        W[e] = h.elen[e] * h.edist[e];
        invd[e] = 1.0 / h.edist[e];
    }
    for (int e = 0; e < h.nce; ++e) ctw[e] = h.celen[e] / h.cedist[e];
    m->a.upload(h.a, s); m->ac.upload(h.ac, s);
    m->elam.upload(h.elam, s); m->etw.upload(tw, s); m->eW.upload(W, s);
    m->einvd.upload(invd, s); m->elen.upload(h.elen, s);
    m->cetw.upload(ctw, s); m->celam.upload(h.celam, s);
    m->fo_w.upload(h.fo_w, s); m->co_w.upload(h.co_w, s); m->cr_w.upload(h.cr_w, s);
    m->eK.upload(h.eK, s); m->eL.upload(h.eL, s); m->erK.upload(h.erK, s); m->erL.upload(h.erL, s);
    m->ceI.upload(h.ceI, s); m->ceJ.upload(h.ceJ, s);
    m->cf_edge.upload(h.cf_edge, s); m->cf_nb.upload(h.cf_nb, s);
    m->fo_c.upload(h.fo_c, s); m->co_f.upload(h.co_f, s); m->cr_e.upload(h.cr_e, s);
    {
        std::vector<int> ck(h.cr_e.size(), 0), cl(h.cr_e.size(), 0);
        std::vector<double> cg(h.cr_e.size(), 0.0), cg2(h.cr_e.size(), 0.0);
        for (size_t q = 0; q < h.cr_e.size(); ++q) {
            const int e = h.cr_e[q];
            if (e < 0) continue;
            ck[q] = h.eK[e];
            cl[q] = h.eL[e];
            cg[q] = 0.5 * h.cr_w[q] * invd[e];
            cg2[q] = 0.5 * h.cr_w[q] * invd[e] * invd[e];
        }
        m->cr_k.upload(ck, s); m->cr_l.upload(cl, s); m->cr_g.upload(cg, s); m->cr_g2.upload(cg2, s);
    }
    {
        // fine-cell edge slots resolved: density sides, lambda, 0.5 |e| / d_e, tw_e
        const size_t nq = h.cf_edge.size();
        std::vector<int> rk(nq, 0), rl(nq, 0);
        std::vector<double> lam(nq, 0.0), bw(nq, 0.0), tws(nq, 0.0);
        for (size_t q = 0; q < nq; ++q) {
            const int e = h.cf_edge[q];
            if (e < 0) continue;
            rk[q] = h.erK[e];
            rl[q] = h.erL[e];
            lam[q] = h.elam[e];
            bw[q] = 0.5 * h.elen[e] * invd[e];
            tws[q] = tw[e];
        }
        m->cf_rk.upload(rk, s); m->cf_rl.upload(rl, s);
        m->cf_lam.upload(lam, s); m->cf_bw.upload(bw, s); m->cf_tw.upload(tws, s);
    }
    m->cc_edge.upload(h.cc_edge, s); m->cc_nb.upload(h.cc_nb, s);
    m->color.upload(h.color, s);
    m->slv.clear();
    for (size_t l = 0; l < h.slevels.size(); ++l) {
        const SLevelHost &L = h.slevels[l];
        SLevelDev D;
        D.n = L.n; D.w = L.w; D.ncolor = L.ncolor;
        D.nbr.upload(L.nbr, s);
        if (!L.color.empty()) { D.color.upload(L.color, s); D.slot_of.upload(L.slot_of, s); }
        if (!L.agg.empty()) {
            D.n_next = (int)L.mem_ptr.size() - 1;
            D.agg.upload(L.agg, s); D.mem_ptr.upload(L.mem_ptr, s); D.mem_idx.upload(L.mem_idx, s);
        }
        m->slv.push_back(std::move(D));
    }
    m->lv.clear();
    for (size_t l = 0; l < h.levels.size(); ++l) {
        const MGLevelHost &L = h.levels[l];
        MGLevelDev D;
        D.n = L.n; D.ne = L.ne; D.w = L.w;
        D.nb.upload(L.nb, s); D.ed.upload(L.ed, s);
        if (!L.agg.empty()) {
            D.n_next = (int)L.mem_ptr.size() - 1;
            D.ne_next = (int)L.cedge_ptr.size() - 1;
            D.agg.upload(L.agg, s); D.mem_ptr.upload(L.mem_ptr, s); D.mem_idx.upload(L.mem_idx, s);
            D.cedge_ptr.upload(L.cedge_ptr, s); D.cedge_idx.upload(L.cedge_idx, s);
        }
        m->lv.push_back(std::move(D));
    }
    OT_HIP(hipStreamSynchronize(s));
}

}  // namespace otbb
