// Host-only inspection of the structured mesh generator and its derived
// structures (no device call), so that host logic can be checked on
// machines without a GPU.
#include <cstring>

#include "../../include/otbb_debug.h"
#include "mesh.hpp"

using namespace otbb;

namespace otbb {
void derive_host_only(MeshHost &h);
}

namespace {
template <typename F>
int guard_dbg(F &&f) {
    try {
        f();
        return OT_OK;
    } catch (const OtError &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return OT_EINVAL;
    }
}
}  // namespace

extern "C" {

int otbb_debug_structured_sizes(int32_t n, int32_t cartesian, int32_t out[8]) {
    return guard_dbg([&] {
        OT_REQUIRE(out, OT_EINVAL, "null argument");
        MeshHost h;
        if (cartesian == 3) cartesian3d_desc(n, h);
        else structured_desc(n, cartesian != 0, h);
        derive_host_only(h);
        out[0] = h.nf; out[1] = h.nc; out[2] = h.ne; out[3] = h.nce;
        out[4] = (int32_t)h.ov_f.size(); out[5] = (int32_t)h.levels.size(); out[6] = h.ncolor; out[7] = h.wf;
    });
}

int otbb_debug_structured_arrays(int32_t n, int32_t cartesian, int32_t *fe_cell, int32_t *fe_rho,
                                 double *fe_len, double *fe_dist, double *fe_lambda, int32_t *ov_fine,
                                 int32_t *ov_coarse, double *ov_area, int32_t *ce_cell, double *ce_len,
                                 double *ce_dist, int32_t *color) {
    return guard_dbg([&] {
        MeshHost h;
        if (cartesian == 3) cartesian3d_desc(n, h);
        else structured_desc(n, cartesian != 0, h);
        derive_host_only(h);
        for (int e = 0; e < h.ne; ++e) {
            if (fe_cell) { fe_cell[2 * e] = h.eK[e]; fe_cell[2 * e + 1] = h.eL[e]; }
            if (fe_rho) { fe_rho[2 * e] = h.erK[e]; fe_rho[2 * e + 1] = h.erL[e]; }
            if (fe_len) fe_len[e] = h.elen[e];
            if (fe_dist) fe_dist[e] = h.edist[e];
            if (fe_lambda) fe_lambda[e] = h.elam[e];
        }
        for (size_t t = 0; t < h.ov_f.size(); ++t) {
            if (ov_fine) ov_fine[t] = h.ov_f[t];
            if (ov_coarse) ov_coarse[t] = h.ov_c[t];
            if (ov_area) ov_area[t] = h.ov_a[t];
        }
        for (int e = 0; e < h.nce; ++e) {
            if (ce_cell) { ce_cell[2 * e] = h.ceI[e]; ce_cell[2 * e + 1] = h.ceJ[e]; }
            if (ce_len) ce_len[e] = h.celen[e];
            if (ce_dist) ce_dist[e] = h.cedist[e];
        }
        if (color) std::memcpy(color, h.color.data(), h.nc * sizeof(int32_t));
    });
}

int otbb_debug_validate_desc(const ot_mesh_desc *d) {
    return guard_dbg([&] {
        OT_REQUIRE(d, OT_EINVAL, "null argument");
        MeshHost h;
        h.nf = d->n_fine; h.nc = d->n_coarse; h.ne = d->n_fedge; h.nce = d->n_cedge;
        OT_REQUIRE(h.nf > 0 && h.nc > 0 && h.ne >= 0 && h.nce >= 0 && d->n_overlap >= 0, OT_EINVAL, "bad sizes");
        h.a.assign(d->fine_area, d->fine_area + h.nf);
        h.ac.assign(d->coarse_area, d->coarse_area + h.nc);
        h.ov_f.assign(d->ov_fine, d->ov_fine + d->n_overlap);
        h.ov_c.assign(d->ov_coarse, d->ov_coarse + d->n_overlap);
        h.ov_a.assign(d->ov_area, d->ov_area + d->n_overlap);
        for (int e = 0; e < h.ne; ++e) {
            h.eK.push_back(d->fe_cell[2 * e]); h.eL.push_back(d->fe_cell[2 * e + 1]);
            h.erK.push_back(d->fe_rho[2 * e]); h.erL.push_back(d->fe_rho[2 * e + 1]);
        }
        h.elen.assign(d->fe_len, d->fe_len + h.ne);
        h.edist.assign(d->fe_dist, d->fe_dist + h.ne);
        h.elam.assign(d->fe_lambda, d->fe_lambda + h.ne);
        for (int e = 0; e < h.nce; ++e) { h.ceI.push_back(d->ce_cell[2 * e]); h.ceJ.push_back(d->ce_cell[2 * e + 1]); }
        h.celen.assign(d->ce_len, d->ce_len + h.nce);
        h.cedist.assign(d->ce_dist, d->ce_dist + h.nce);
        h.celam.assign(d->ce_lambda, d->ce_lambda + h.nce);
        derive_host_only(h);
    });
}

}  // extern "C"

extern "C" int otbb_debug_schur_levels(int32_t n, int32_t cartesian, int32_t *out, int32_t cap) {
    return guard_dbg([&] {
        OT_REQUIRE(out && cap >= 1, OT_EINVAL, "null argument");
        MeshHost h;
        structured_desc(n, cartesian != 0, h);
        derive_host_only(h);
        int nl = (int)h.slevels.size();
        out[0] = nl;
        for (int l = 0; l < nl && 1 + 3 * l + 2 < cap; ++l) {
            out[1 + 3 * l] = h.slevels[l].n;
            out[2 + 3 * l] = h.slevels[l].w;
            out[3 + 3 * l] = h.slevels[l].ncolor;
        }
    });
}
