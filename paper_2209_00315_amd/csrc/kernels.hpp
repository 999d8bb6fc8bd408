// Device kernels of the otbb library (gfx950, wave64).
//
// Index conventions: fine cell i in [0, nf), potential level k in [0, K]
// (the paper's levels 1..K+1), coarse cell j in [0, nc), density level k in
// [0, K) (the paper's 1..K).  Density "time indices" L in [0, K+1] address
// (rho_in, rho^1..rho^K, rho_f).  Potential level k sits between density
// indices L = k and L = k + 1.  All per-slice topology arrays are ELL,
// column-major (t * n + cell), padded with -1; they are the same for every
// time slice, so one launch covers all slices (blockIdx.y = slice) and the
// topology is read from cache after the first slice.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

namespace otbb {
namespace kern {

constexpr int BS = 256;

struct MeshView {
    int nf, nc, ne, nce, wf, wo, woc, wr, wcc;
    const double *a, *ac, *elam, *etw, *eW, *einvd, *elen, *cetw, *celam, *fo_w, *co_w, *cr_w;
    const int *eK, *eL, *erK, *erL, *ceI, *ceJ, *cf_edge, *cf_nb, *fo_c, *co_f, *cr_e, *cc_edge, *cc_nb;
    const int *cr_k, *cr_l;     // R_T slots resolved: potential cells of the edge
    const double *cr_g;         // R_T slots resolved: 0.5 cr_w / d_e
    const double *cr_g2;        // R_T slots resolved: 0.5 cr_w / d_e^2
    // fine-cell edge slots resolved (slot t of cell i, [t nf + i]): density
    // sides of the edge, lambda, 0.5 |e| / d_e, tw_e
    const int *cf_rk, *cf_rl;
    const double *cf_lam, *cf_bw, *cf_tw;
};

struct StateView {
    int K;
    double dt, area;
    const double *phi, *rho, *s, *rin, *rf;
};

// ------------------------------------------------------------ XCD locality
// The dispatcher places workgroup b (linear id) on XCD b % 8, and each XCD
// has its own L2.  For a grid row of gx blocks (gx % 8 == 0, so block
// (x, y) sits on XCD x % 8 for every row y), this renumbers x so that every
// XCD takes one contiguous band of gx / 8 blocks: cells with nearby indices
// then share an L2, and the halos of gathered neighbour data are fetched
// by one XCD instead of by two at every block boundary.  Any other gx keeps
// the identity.
__device__ __forceinline__ int xcd_band_block() {
    const int gx = gridDim.x, bx = blockIdx.x;
    return (gx & 7) ? bx : (bx & 7) * (gx >> 3) + (bx >> 3);
}

// ---------------------------------------------------------------- reductions
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[BS / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    v = (threadIdx.x < BS / 64) ? sh[threadIdx.x] : 0.0;
    if (wid == 0) v = wave_sum(v);
    return v;
}

__device__ __forceinline__ double block_min(double v) {
    __shared__ double sh[BS / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    v = (threadIdx.x < BS / 64) ? sh[threadIdx.x] : DBL_MAX;
    if (wid == 0) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    }
    return v;
}

// out[seg] = sum_b part[seg * nblk + b]   (one block per segment)
__global__ void k_seg_final(const double *__restrict__ part, int nblk, double *__restrict__ out) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += BS) v += part[(size_t)blockIdx.x * nblk + b];
    v = block_sum(v);
    if (threadIdx.x == 0) out[blockIdx.x] = v;
}

__global__ void k_min_final(const double *__restrict__ part, int nblk, double *__restrict__ out) {
    double v = DBL_MAX;
    for (int b = threadIdx.x; b < nblk; b += BS) v = fmin(v, part[b]);
    v = block_min(v);
    if (threadIdx.x == 0) out[0] = v;
}

// Segmented (weighted) sums: part[seg * nblk + b] over x[seg * n + i] * w[i].
template <typename T>
__global__ void k_seg_partial(const T *__restrict__ x, const double *__restrict__ w, int n,
                              double *__restrict__ part) {
    const int seg = blockIdx.y;
    double v = 0.0;
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) {
        double xi = (double)x[(size_t)seg * n + i];
        v += w ? w[i] * xi : xi;
    }
    v = block_sum(v);
    if (threadIdx.x == 0) part[(size_t)seg * gridDim.x + blockIdx.x] = v;
}

// Segmented dot products: part[seg * nblk + b] of sum_i x * y over segment seg.
template <typename T>
__global__ void k_seg_dot_partial(const T *__restrict__ x, const T *__restrict__ y, int n,
                                  double *__restrict__ part) {
    const int seg = blockIdx.y;
    double v = 0.0;
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) {
        size_t q = (size_t)seg * n + i;
        v += (double)x[q] * (double)y[q];
    }
    v = block_sum(v);
    if (threadIdx.x == 0) part[(size_t)seg * gridDim.x + blockIdx.x] = v;
}

// ----------------------------------------------------------- state helpers
__device__ __forceinline__ double rho_at(const StateView &S, int nc, int L, int j) {
    return L == 0 ? S.rin[j] : (L == S.K + 1 ? S.rf[j] : S.rho[(size_t)(L - 1) * nc + j]);
}

// rho~ on fine edge e at potential level k: R_E((rho^L + rho^{L+1})/2), L = k
__device__ __forceinline__ double rho_edge(const MeshView &m, const StateView &S, int k, int e) {
    const int rK = m.erK[e], rL = m.erL[e];
    const double lam = m.elam[e];
    const double mK = 0.5 * (rho_at(S, m.nc, k, rK) + rho_at(S, m.nc, k + 1, rK));
    const double mL = 0.5 * (rho_at(S, m.nc, k, rL) + rho_at(S, m.nc, k + 1, rL));
    return lam * mK + (1.0 - lam) * mL;
}

__device__ __forceinline__ double grad_phi(const MeshView &m, const double *ph, int e) {
    return (ph[m.eK[e]] - ph[m.eL[e]]) * m.einvd[e];
}

// ------------------------------------------------------------- residual F
// F_phi^k = -Omega (rho^{k+1} - rho^k)/dt + sum_e tw rho~ (phi_i - phi_nb)
__global__ void k_res_phi(MeshView m, StateView S, double *__restrict__ F, double *__restrict__ part) {
    const int i = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    double sq = 0.0;
    if (i < m.nf) {
        const double *ph = S.phi + (size_t)k * m.nf;
        double v = 0.0;
        for (int t = 0; t < m.wo; ++t) {
            const int c = m.fo_c[t * m.nf + i];
            if (c < 0) break;
            v -= m.fo_w[t * m.nf + i] * (rho_at(S, m.nc, k + 1, c) - rho_at(S, m.nc, k, c)) / S.dt;
        }
        const double pi = ph[i];
        for (int t = 0; t < m.wf; ++t) {
            const int e = m.cf_edge[t * m.nf + i];
            if (e < 0) break;
            v += m.etw[e] * rho_edge(m, S, k, e) * (pi - ph[m.cf_nb[t * m.nf + i]]);
        }
        F[(size_t)k * m.nf + i] = v;
        sq = v * v;
    }
    sq = block_sum(sq);
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = sq;
}

// F_rho^k = Omega^T (phi^{k+1} - phi^k)/dt + 1/4 R_T(g_k^2 + g_{k+1}^2) + a' s;  F_s = rho s - mu
__global__ void k_res_rho(MeshView m, StateView S, double mu, double *__restrict__ Frho,
                          double *__restrict__ Fs, double *__restrict__ part) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    double sq = 0.0;
    if (j < m.nc) {
        const double *p0 = S.phi + (size_t)k * m.nf, *p1 = p0 + m.nf;
        double v = 0.0;
        for (int t = 0; t < m.woc; ++t) {
            const int f = m.co_f[t * m.nc + j];
            if (f < 0) break;
            v += m.co_w[t * m.nc + j] * (p1[f] - p0[f]) / S.dt;
        }
        double hj = 0.0;
        for (int t = 0; t < m.wr; ++t) {
            const int e = m.cr_e[t * m.nc + j];
            if (e < 0) break;
            const double g0 = grad_phi(m, p0, e), g1 = grad_phi(m, p1, e);
            hj += m.cr_w[t * m.nc + j] * (g0 * g0 + g1 * g1);
        }
        const size_t q = (size_t)k * m.nc + j;
        v += 0.25 * hj + m.ac[j] * S.s[q];
        const double fs = S.rho[q] * S.s[q] - mu;
        Frho[q] = v;
        Fs[q] = fs;
        sq = v * v + fs * fs;
    }
    sq = block_sum(sq);
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = sq;
}

// ------------------------------------------------------ saddle operator J_P
// value of (P^T x_rho) at density level l (0-based), zero outside [0, K)
__device__ __forceinline__ double ptx_at(const double *xr, const double *cs, double area, int K, int nc,
                                         int l, int j) {
    return (l >= 0 && l < K) ? xr[(size_t)l * nc + j] - cs[l] / area : 0.0;
}

// y_phi^k = A^k x_phi^k + (B^T w)^k with w = P^T x_rho, cs[l] = a'^T x_rho^l:
// (B^T w)^k = Omega (w^{k-1} - w^k)/dt + 1/2 sum_e sgn len g_e R_E(w^{k-1} + w^k)_e
// xphi == nullptr drops the A^k x_phi^k term (y = B^T P^T x_rho); dscale !=
// nullptr divides the result by it (entries 0 leave it unscaled), as
// k_dscale with inv = 1 would in a second pass.
__global__ void k_saddle_phi(MeshView m, StateView S, const double *__restrict__ xphi,
                             const double *__restrict__ xr, const double *__restrict__ cs,
                             const double *__restrict__ dscale, double *__restrict__ y) {
    const int i = xcd_band_block() * BS + threadIdx.x, k = blockIdx.y;
    if (i >= m.nf) return;
    const int K = S.K, nc = m.nc;
    const double *xp = xphi ? xphi + (size_t)k * m.nf : nullptr;
    const double *ph = S.phi + (size_t)k * m.nf;
    const double xi = xp ? xp[i] : 0.0;
    double v = 0.0;
    const double phi_i = ph[i];
    for (int t = 0; t < m.wf; ++t) {
        const int q = t * m.nf + i;
        if (m.cf_edge[q] < 0) break;
        const int nb = m.cf_nb[q];
        const int rK = m.cf_rk[q], rL = m.cf_rl[q];
        const double lam = m.cf_lam[q];
        if (xp) {
            const double mK = 0.5 * (rho_at(S, nc, k, rK) + rho_at(S, nc, k + 1, rK));
            const double mL = 0.5 * (rho_at(S, nc, k, rL) + rho_at(S, nc, k + 1, rL));
            v += m.cf_tw[q] * (lam * mK + (1.0 - lam) * mL) * (xi - xp[nb]);
        }
        // sgn_e (grad phi)_e = (phi_i - phi_nb) / d_e whichever side i is on
        const double wK = ptx_at(xr, cs, S.area, K, nc, k - 1, rK) + ptx_at(xr, cs, S.area, K, nc, k, rK);
        const double wL = ptx_at(xr, cs, S.area, K, nc, k - 1, rL) + ptx_at(xr, cs, S.area, K, nc, k, rL);
        v += m.cf_bw[q] * (phi_i - ph[nb]) * (lam * wK + (1.0 - lam) * wL);
    }
    for (int t = 0; t < m.wo; ++t) {
        const int c = m.fo_c[t * m.nf + i];
        if (c < 0) break;
        v += m.fo_w[t * m.nf + i] *
             (ptx_at(xr, cs, S.area, K, nc, k - 1, c) - ptx_at(xr, cs, S.area, K, nc, k, c)) / S.dt;
    }
    const size_t q = (size_t)k * m.nf + i;
    if (dscale) {
        const double di = dscale[q];
        v *= di != 0.0 ? 1.0 / di : 1.0;
    }
    y[q] = v;
}

// u^k = (B x_phi)^k - cfac C (P^T x_rho)^k  (C = a' s / rho); cfac = 0 drops C.
// (B x)^k = Omega^T (x^{k+1} - x^k)/dt + 1/2 sum R_T-weights (g^k grad x^k + g^{k+1} grad x^{k+1})
// Writes u and per-block partial slice sums of u (for the projector P).
__global__ void k_opB(MeshView m, StateView S, const double *__restrict__ xphi,
                      const double *__restrict__ xr, const double *__restrict__ cs, double cfac,
                      double *__restrict__ u, double *__restrict__ part) {
    const int j = xcd_band_block() * BS + threadIdx.x, k = blockIdx.y;
    double v = 0.0;
    if (j < m.nc) {
        const double *x0 = xphi + (size_t)k * m.nf, *x1 = x0 + m.nf;
        const double *p0 = S.phi + (size_t)k * m.nf, *p1 = p0 + m.nf;
        for (int t = 0; t < m.woc; ++t) {
            const int f = m.co_f[t * m.nc + j];
            if (f < 0) break;
            v += m.co_w[t * m.nc + j] * (x1[f] - x0[f]) / S.dt;
        }
        for (int t = 0; t < m.wr; ++t) {
            const int q = t * m.nc + j;
            if (m.cr_e[q] < 0) break;
            const int eK = m.cr_k[q], eL = m.cr_l[q];
            v += m.cr_g2[q] * ((p0[eK] - p0[eL]) * (x0[eK] - x0[eL]) + (p1[eK] - p1[eL]) * (x1[eK] - x1[eL]));
        }
        const size_t q = (size_t)k * m.nc + j;
        if (cfac != 0.0) v -= cfac * m.ac[j] * S.s[q] / S.rho[q] * ptx_at(xr, cs, S.area, S.K, m.nc, k, j);
        u[q] = v;
    }
    v = block_sum(v);
    if (part && threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = v;
}

// y_rho^k -= a' us[k] / area   (the projector P)
template <typename T>
__global__ void k_proj_fix(const double *__restrict__ ac, int nc, const double *__restrict__ us,
                           double area, T *__restrict__ y) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (j < nc) y[(size_t)k * nc + j] -= (T)(ac[j] * us[k] / area);
}

// diagonal of C = M' Diag(rho)^-1 Diag(s): c[k nc + j] = a'_j s / rho
__global__ void k_c_diag(int nc, const double *__restrict__ ac, StateView S, double *__restrict__ c) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (j >= nc) return;
    const size_t q = (size_t)k * nc + j;
    c[q] = ac[j] * S.s[q] / S.rho[q];
}

// x += alpha p; r -= alpha q (the two CG updates in one pass)
__global__ void k_cg_update(size_t n, double alpha, const double *__restrict__ p, const double *__restrict__ q,
                            double *__restrict__ x, double *__restrict__ r) {
    for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) {
        x[i] = alpha * p[i] + 1.0 * x[i];
        r[i] = -alpha * q[i] + 1.0 * r[i];
    }
}

// w^k = r^k - a' lam[k]
__global__ void k_sub_slice_cols(int nc, const double *__restrict__ ac, const double *__restrict__ lam,
                                 const double *__restrict__ r, double *__restrict__ w) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (j < nc) {
        const size_t q = (size_t)k * nc + j;
        w[q] = r[q] - ac[j] * lam[k];
    }
}

// y = M x for a small dense n x n matrix M (row-major); one block
__global__ void k_small_gemv(int n, const double *__restrict__ M, const double *__restrict__ x,
                             double *__restrict__ y) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double v = 0.0;
        for (int l = 0; l < n; ++l) v += M[(size_t)i * n + l] * x[l];
        y[i] = v;
    }
}

// y^k -= sums[k] * scale   (P^T or mean removal)
template <typename T>
__global__ void k_slice_shift(int n, const double *__restrict__ sums, double scale, T *__restrict__ y) {
    const int i = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (i < n) y[(size_t)k * n + i] -= (T)(sums[k] * scale);
}

// ------------------------------------------------------- vector utilities
template <typename T>
__global__ void k_fill(T *__restrict__ x, size_t n, T v) {
    for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) x[i] = v;
}

template <typename TO, typename TI>
__global__ void k_convert(const TI *__restrict__ x, TO *__restrict__ y, size_t n) {
    for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) y[i] = (TO)x[i];
}

// y = a x + b y
template <typename T>
__global__ void k_axpby(size_t n, double a, const T *__restrict__ x, double b, T *__restrict__ y) {
    // b == 0 overwrites y without reading it: y may be uninitialised memory,
    // whose NaN bit patterns would survive a multiplication by zero.
    for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS)
        y[i] = (T)(b == 0.0 ? a * (double)x[i] : a * (double)x[i] + b * (double)y[i]);
}

// partial sums of squares
template <typename T>
__global__ void k_nrm2_partial(size_t n, const T *__restrict__ x, double *__restrict__ part) {
    double v = 0.0;
    for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) {
        double xi = (double)x[i];
        v += xi * xi;
    }
    v = block_sum(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// Multi-dot for classical Gram-Schmidt: part[v * nblk + b] = sum over the
// block's rows of V_v . w for the group of vectors v = g*8 .. g*8+7.
template <typename T>
__global__ void k_multidot(size_t n, const T *__restrict__ V, size_t ldv, int nv, const T *__restrict__ w,
                           double *__restrict__ part) {
    const int g0 = blockIdx.y * 8;
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) {
        const double wi = (double)w[i];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (g0 + q < nv) acc[q] += (double)V[(size_t)(g0 + q) * ldv + i] * wi;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (g0 + q >= nv) break;
        double s = block_sum(acc[q]);
        if (threadIdx.x == 0) part[(size_t)(g0 + q) * gridDim.x + blockIdx.x] = s;
    }
}

// w -= sum_v h[v] V_v, then partial sums of |w|^2 (h on device)
template <typename T>
__global__ void k_gs_update(size_t n, const T *__restrict__ V, size_t ldv, int nv, const double *__restrict__ h,
                            T *__restrict__ w, double *__restrict__ part) {
    double sq = 0.0;
    for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) {
        double wi = (double)w[i];
#pragma unroll 8
        for (int v = 0; v < nv; ++v) wi -= h[v] * (double)V[(size_t)v * ldv + i];
        const T wt = (T)wi;
        w[i] = wt;
        sq += (double)wt * (double)wt;
    }
    sq = block_sum(sq);
    if (threadIdx.x == 0) part[blockIdx.x] = sq;
}

// x += sum_v y[v] Z_v  (or x = ... when beta = 0)
template <typename T, typename TX>
__global__ void k_combine(size_t n, const T *__restrict__ Z, size_t ldz, int nv, const double *__restrict__ y,
                          double beta, TX *__restrict__ x) {
    for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) {
        double v = beta == 0.0 ? 0.0 : beta * (double)x[i];
        for (int q = 0; q < nv; ++q) v += y[q] * (double)Z[(size_t)q * ldz + i];
        x[i] = (TX)v;
    }
}

// ------------------------------------------ preconditioner (type T) pieces
// Per-linearisation coefficient arrays (type T):
//   g[k][e]   gradient of the current phi at potential level k
//   w0[k][e]  tw_e rho~^k_e   (level-0 multigrid edge weights)
//   wc[k][ce] coarse edge weights of A~^k: len'/dist' (lam' rho_I + (1-lam') rho_J)
template <typename T>
__global__ void k_lin_edges(MeshView m, StateView S, T *__restrict__ g, T *__restrict__ w0) {
    const int e = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (e >= m.ne) return;
    const double *ph = S.phi + (size_t)k * m.nf;
    g[(size_t)k * m.ne + e] = (T)grad_phi(m, ph, e);
    w0[(size_t)k * m.ne + e] = (T)(m.etw[e] * rho_edge(m, S, k, e));
}

template <typename T>
__global__ void k_lin_cedges(MeshView m, StateView S, T *__restrict__ wc) {
    const int e = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (e >= m.nce) return;
    const double *r = S.rho + (size_t)k * m.nc;
    const double lam = m.celam[e];
    wc[(size_t)k * m.nce + e] = (T)(m.cetw[e] * (lam * r[m.ceI[e]] + (1.0 - lam) * r[m.ceJ[e]]));
}

// Pseudo-Schur pass 1: u^k_i = (J (z^{k-1} + z^k)/2)_i = sum_c Omega_ic (..)_c / a_i
template <typename T>
__global__ void k_schur_lift(MeshView m, int K, const T *__restrict__ z, T *__restrict__ u) {
    const int i = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (i >= m.nf) return;
    double v = 0.0;
    for (int t = 0; t < m.wo; ++t) {
        const int c = m.fo_c[t * m.nf + i];
        if (c < 0) break;
        double zz = 0.0;
        if (k >= 1) zz += (double)z[(size_t)(k - 1) * m.nc + c];
        if (k < K) zz += (double)z[(size_t)k * m.nc + c];
        v += m.fo_w[t * m.nf + i] * 0.5 * zz;
    }
    u[(size_t)k * m.nf + i] = (T)(v / m.a[i]);
}

// Pseudo-Schur pass 2: v^k = M^-1 B~ z at potential level k:
//   B~ z = Omega (z^k - z^{k-1})/dt + R_Tf[g^k * grad u^k]
template <typename T>
__global__ void k_schur_btilde(MeshView m, int K, double dt, const T *__restrict__ z, const T *__restrict__ u,
                               const T *__restrict__ g, T *__restrict__ v) {
    const int i = xcd_band_block() * BS + threadIdx.x, k = blockIdx.y;
    if (i >= m.nf) return;
    double acc = 0.0;
    for (int t = 0; t < m.wo; ++t) {
        const int c = m.fo_c[t * m.nf + i];
        if (c < 0) break;
        double dz = 0.0;
        if (k < K) dz += (double)z[(size_t)k * m.nc + c];
        if (k >= 1) dz -= (double)z[(size_t)(k - 1) * m.nc + c];
        acc += m.fo_w[t * m.nf + i] * dz / dt;
    }
    const T *uk = u + (size_t)k * m.nf;
    const T *gk = g + (size_t)k * m.ne;
    const double ui = (double)uk[i];
    for (int t = 0; t < m.wf; ++t) {
        const int e = m.cf_edge[t * m.nf + i];
        if (e < 0) break;
        const int nb = m.cf_nb[t * m.nf + i];
        const bool isK = m.eK[e] == i;
        const double side = isK ? m.elam[e] : 1.0 - m.elam[e];
        const double du = (isK ? 1.0 : -1.0) * (ui - (double)uk[nb]) * m.einvd[e];   // (u_K - u_L)/d
        acc += side * m.eW[e] * (double)gk[e] * du;
    }
    v[(size_t)k * m.nf + i] = (T)(acc / m.a[i]);
}

// Pseudo-Schur pass 3: out^k = s (A~ z)^k - rho (B v)^k
template <typename T>
__global__ void k_schur_out(MeshView m, int K, double dt, const T *__restrict__ z, const T *__restrict__ v,
                            const T *__restrict__ g, const T *__restrict__ wc, const T *__restrict__ rhoT,
                            const T *__restrict__ sT, T *__restrict__ out) {
    const int j = xcd_band_block() * BS + threadIdx.x, k = blockIdx.y;
    if (j >= m.nc) return;
    const size_t q = (size_t)k * m.nc + j;
    const T *zk = z + (size_t)k * m.nc;
    const T *wck = wc + (size_t)k * m.nce;
    double at = 0.0;
    const double zj = (double)zk[j];
    for (int t = 0; t < m.wcc; ++t) {
        const int e = m.cc_edge[t * m.nc + j];
        if (e < 0) break;
        at += (double)wck[e] * (zj - (double)zk[m.cc_nb[t * m.nc + j]]);
    }
    const T *v0 = v + (size_t)k * m.nf, *v1 = v0 + m.nf;
    const T *g0 = g + (size_t)k * m.ne, *g1 = g0 + m.ne;
    double b = 0.0;
    for (int t = 0; t < m.woc; ++t) {
        const int f = m.co_f[t * m.nc + j];
        if (f < 0) break;
        b += m.co_w[t * m.nc + j] * ((double)v1[f] - (double)v0[f]) / dt;
    }
    for (int t = 0; t < m.wr; ++t) {
        const int q = t * m.nc + j;
        const int e = m.cr_e[q];
        if (e < 0) break;
        const int eK = m.cr_k[q], eL = m.cr_l[q];
        b += m.cr_g[q] *
             ((double)g0[e] * ((double)v0[eK] - (double)v0[eL]) + (double)g1[e] * ((double)v1[eK] - (double)v1[eL]));
    }
    out[q] = (T)((double)sT[q] * at - (double)rhoT[q] * b);
}

// Time-blocked forms of passes 2 and 3: one thread per cell and kb
// consecutive time levels.  The cell's stencil (indices and FP64 geometric
// weights) is loaded once into registers instead of once per level, and the
// operand of level k+1 that the next level reads as its level-k operand is
// carried over instead of reloaded.  Used when the mesh's ELL widths fit the
// register caps below (the structured grids do: w_f <= 4, w_o <= 2,
// w_oc <= 3, w_r <= 6, w_cc <= 3); otherwise the per-level kernels above run.
constexpr int kTbWF = 4, kTbWO = 2, kTbWOC = 4, kTbWR = 8, kTbWCC = 4;

template <typename T>
__global__ void __launch_bounds__(BS) k_schur_btilde_tb(MeshView m, int K, int kb, double dt, const T *__restrict__ z,
                                                        const T *__restrict__ u, const T *__restrict__ g,
                                                        T *__restrict__ v) {
    const int i = xcd_band_block() * BS + threadIdx.x;
    if (i >= m.nf) return;
    const int k0 = blockIdx.y * kb, k1 = min(K + 1, k0 + kb);
    int oc[kTbWO];
    double ow[kTbWO];
#pragma unroll
    for (int t = 0; t < kTbWO; ++t) {
        const int c = t < m.wo ? m.fo_c[t * m.nf + i] : -1;
        oc[t] = c >= 0 ? c : 0;
        ow[t] = c >= 0 ? m.fo_w[t * m.nf + i] / dt : 0.0;
    }
    int fe[kTbWF], fn[kTbWF];
    double fw[kTbWF];
#pragma unroll
    for (int t = 0; t < kTbWF; ++t) {
        const int e = t < m.wf ? m.cf_edge[t * m.nf + i] : -1;
        fe[t] = e >= 0 ? e : 0;
        fn[t] = e >= 0 ? m.cf_nb[t * m.nf + i] : i;
        double w = 0.0;
        if (e >= 0) {
            const bool isK = m.eK[e] == i;
            const double side = isK ? m.elam[e] : 1.0 - m.elam[e];
            w = (isK ? 1.0 : -1.0) * side * m.eW[e] * m.einvd[e];
        }
        fw[t] = w;
    }
    const double inva = 1.0 / m.a[i];
    // z at level k-1 for the first level of the block
    T zp[kTbWO];
#pragma unroll
    for (int t = 0; t < kTbWO; ++t) zp[t] = k0 >= 1 ? z[(size_t)(k0 - 1) * m.nc + oc[t]] : (T)0;
    for (int k = k0; k < k1; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < kTbWO; ++t) {
            const T zc = k < K ? z[(size_t)k * m.nc + oc[t]] : (T)0;
            acc += ow[t] * ((double)zc - (double)zp[t]);
            zp[t] = zc;
        }
        const T *uk = u + (size_t)k * m.nf;
        const T *gk = g + (size_t)k * m.ne;
        const double ui = (double)uk[i];
#pragma unroll
        for (int t = 0; t < kTbWF; ++t) acc += fw[t] * (double)gk[fe[t]] * (ui - (double)uk[fn[t]]);
        v[(size_t)k * m.nf + i] = (T)(acc * inva);
    }
}

template <typename T>
__global__ void __launch_bounds__(BS) k_schur_out_tb(MeshView m, int K, int kb, double dt, const T *__restrict__ z,
                                                     const T *__restrict__ v, const T *__restrict__ g,
                                                     const T *__restrict__ wc, const T *__restrict__ rhoT,
                                                     const T *__restrict__ sT, T *__restrict__ out) {
    const int j = xcd_band_block() * BS + threadIdx.x;
    if (j >= m.nc) return;
    const int k0 = blockIdx.y * kb, k1 = min(K, k0 + kb);
    int ce[kTbWCC], cn[kTbWCC];
    bool cv[kTbWCC];
#pragma unroll
    for (int t = 0; t < kTbWCC; ++t) {
        const int e = t < m.wcc ? m.cc_edge[t * m.nc + j] : -1;
        cv[t] = e >= 0;
        ce[t] = cv[t] ? e : 0;
        cn[t] = cv[t] ? m.cc_nb[t * m.nc + j] : j;
    }
    int of[kTbWOC];
    double ow[kTbWOC];
#pragma unroll
    for (int t = 0; t < kTbWOC; ++t) {
        const int f = t < m.woc ? m.co_f[t * m.nc + j] : -1;
        of[t] = f >= 0 ? f : 0;
        ow[t] = f >= 0 ? m.co_w[t * m.nc + j] / dt : 0.0;
    }
    int re[kTbWR], rk[kTbWR], rl[kTbWR];
    double rw[kTbWR];
#pragma unroll
    for (int t = 0; t < kTbWR; ++t) {
        const int q = t * m.nc + j;
        const int e = t < m.wr ? m.cr_e[q] : -1;
        re[t] = e >= 0 ? e : 0;
        rk[t] = e >= 0 ? m.cr_k[q] : 0;
        rl[t] = e >= 0 ? m.cr_l[q] : 0;
        rw[t] = e >= 0 ? m.cr_g[q] : 0.0;
    }
    // operands at level k0 (v and g have K+1 levels)
    T vo[kTbWOC], vk[kTbWR], vl[kTbWR], gg0[kTbWR];
    {
        const T *v0 = v + (size_t)k0 * m.nf;
        const T *g0 = g + (size_t)k0 * m.ne;
#pragma unroll
        for (int t = 0; t < kTbWOC; ++t) vo[t] = v0[of[t]];
#pragma unroll
        for (int t = 0; t < kTbWR; ++t) {
            vk[t] = v0[rk[t]];
            vl[t] = v0[rl[t]];
            gg0[t] = g0[re[t]];
        }
    }
    for (int k = k0; k < k1; ++k) {
        const T *zk = z + (size_t)k * m.nc;
        const T *wck = wc + (size_t)k * m.nce;
        const T *v1 = v + (size_t)(k + 1) * m.nf;
        const T *g1 = g + (size_t)(k + 1) * m.ne;
        const double zj = (double)zk[j];
        double at = 0.0;
#pragma unroll
        for (int t = 0; t < kTbWCC; ++t)
            if (cv[t]) at += (double)wck[ce[t]] * (zj - (double)zk[cn[t]]);
        double b = 0.0;
#pragma unroll
        for (int t = 0; t < kTbWOC; ++t) {
            const T x1 = v1[of[t]];
            b += ow[t] * ((double)x1 - (double)vo[t]);
            vo[t] = x1;
        }
#pragma unroll
        for (int t = 0; t < kTbWR; ++t) {
            const T k1v = v1[rk[t]], l1v = v1[rl[t]], g1v = g1[re[t]];
            b += rw[t] * ((double)gg0[t] * ((double)vk[t] - (double)vl[t]) + (double)g1v * ((double)k1v - (double)l1v));
            vk[t] = k1v;
            vl[t] = l1v;
            gg0[t] = g1v;
        }
        const size_t q = (size_t)k * m.nc + j;
        out[q] = (T)((double)sT[q] * at - (double)rhoT[q] * b);
    }
}

// probe vector: 1 at (k, j) with k % 3 == tc and color[j] == c
template <typename T>
__global__ void k_probe(int nc, const int *__restrict__ color, int tc, int c, T *__restrict__ p) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (j < nc) p[(size_t)k * nc + j] = (T)((k % 3 == tc && color[j] == c) ? 1.0 : 0.0);
}

// scatter a probe response into the three diagonals of the time-line blocks
template <typename T>
__global__ void k_probe_scatter(int nc, int K, const int *__restrict__ color, int tc, int c,
                                const T *__restrict__ r, double *__restrict__ d0, double *__restrict__ dl,
                                double *__restrict__ du) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (j >= nc || color[j] != c) return;
    const size_t q = (size_t)k * nc + j;
    const double val = (double)r[q];
    if (k % 3 == tc) d0[q] = val;
    else if (k >= 1 && (k - 1) % 3 == tc) dl[q] = val;
    else if (k + 1 < K && (k + 1) % 3 == tc) du[q] = val;
}

// Thomas factorisation along time for every coarse cell: inv_dd[k] and
// multipliers l[k] = dl[k] / dd[k-1]; weak pivots fall back to the diagonal.
template <typename T>
__global__ void k_tri_factor(int nc, int K, const double *__restrict__ d0, const double *__restrict__ dl,
                             const double *__restrict__ du, T *__restrict__ inv_dd, T *__restrict__ lm,
                             T *__restrict__ up) {
    const int j = blockIdx.x * BS + threadIdx.x;
    if (j >= nc) return;
    double prev = 0.0, prev_up = 0.0;
    for (int k = 0; k < K; ++k) {
        const size_t q = (size_t)k * nc + j;
        double d = d0[q], l = 0.0;
        if (k > 0 && prev != 0.0) {
            l = dl[q] / prev;
            double dd = d - l * prev_up;
            if (!(fabs(dd) > 1e-3 * fabs(d)) || !isfinite(dd)) { l = 0.0; dd = d; }
            d = dd;
        }
        if (!(fabs(d) > 0.0) || !isfinite(d)) d = 1.0;
        inv_dd[q] = (T)(1.0 / d);
        lm[q] = (T)l;
        const double u = (k + 1 < K) ? du[q] : 0.0;
        up[q] = (T)u;
        prev = d;
        prev_up = u;
    }
}

// Forward/backward substitution along time for every coarse cell.  Loads of
// a chunk of TC levels are issued before the dependent arithmetic so that
// each thread keeps TC memory requests in flight (one thread per cell gives
// only nc threads, so latency hiding has to come from within the thread).
template <typename T, int FINE = 0>
__global__ void k_tri_solve(int nc, int K, const T *__restrict__ inv_dd, const T *__restrict__ lm,
                            const T *__restrict__ up, const T *__restrict__ r, T *__restrict__ x) {
    constexpr int TC = 8;
    const int j = blockIdx.x * BS + threadIdx.x;
    if (j >= nc) return;
    double y = 0.0;
    for (int k0 = 0; k0 < K; k0 += TC) {
        double rr[TC], ll[TC];
#pragma unroll
        for (int t = 0; t < TC; ++t) {
            const int k = k0 + t;
            const size_t q = (size_t)k * nc + j;
            rr[t] = k < K ? (double)r[q] : 0.0;
            ll[t] = k < K ? (double)lm[q] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < TC; ++t) {
            const int k = k0 + t;
            if (k < K) {
                y = rr[t] - ll[t] * y;
                x[(size_t)k * nc + j] = (T)y;
            }
        }
    }
    double xn = 0.0;
    const int kl = ((K + TC - 1) / TC) * TC;
    for (int k0 = kl - TC; k0 >= 0; k0 -= TC) {
        double yy[TC], uu[TC], dd[TC];
#pragma unroll
        for (int t = 0; t < TC; ++t) {
            const int k = k0 + t;
            const size_t q = (size_t)k * nc + j;
            yy[t] = k < K ? (double)x[q] : 0.0;
            uu[t] = k < K ? (double)up[q] : 0.0;
            dd[t] = k < K ? (double)inv_dd[q] : 0.0;
        }
#pragma unroll
        for (int t = TC - 1; t >= 0; --t) {
            const int k = k0 + t;
            if (k < K) {
                xn = (yy[t] - uu[t] * xn) * dd[t];
                x[(size_t)k * nc + j] = (T)xn;
            }
        }
    }
}

// Same solve with one wavefront per cell, one lane per time level: each
// Thomas sweep is a first-order linear recurrence, y_k = a_k y_{k-1} + b_k
// (forward: a = -l, b = r; backward, from the end: x_k = -u_k d_k x_{k+1} +
// d_k y_k), i.e. the composition of affine maps, which a Hillis-Steele scan
// over the 64 lanes evaluates in 6 shuffle steps instead of 64 dependent
// steps.  Lines longer than 64 are done in chunks with the value at the
// chunk edge carried over; y stays in registers (K <= 64 kTriScanChunks).
constexpr int kTriScanChunks = 4;

template <typename T, int FINE = 0>
__global__ void __launch_bounds__(BS) k_tri_scan(int nc, int K, const T *__restrict__ inv_dd,
                                                 const T *__restrict__ lm, const T *__restrict__ up,
                                                 const T *__restrict__ r, T *__restrict__ x) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    if (j >= nc) return;                       // whole wavefront leaves together
    const int nch = (K + 63) / 64;
    double ys[kTriScanChunks];
    double carry = 0.0;
#pragma unroll
    for (int c = 0; c < kTriScanChunks; ++c) {
        if (c >= nch) break;
        const int k = c * 64 + lane;
        const bool in = k < K;
        const size_t q = (size_t)k * nc + j;
        double a = in ? -(double)lm[q] : 1.0;  // identity map on lanes past the line
        double b = in ? (double)r[q] : 0.0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double ap = __shfl_up(a, off, 64), bp = __shfl_up(b, off, 64);
            if (lane >= off) {
                b = a * bp + b;
                a = a * ap;
            }
        }
        const double y = a * carry + b;
        ys[c] = y;
        carry = __shfl(y, 63, 64);
    }
    carry = 0.0;
#pragma unroll
    for (int c = kTriScanChunks - 1; c >= 0; --c) {
        if (c >= nch) continue;
        const int k = c * 64 + lane;
        const bool in = k < K;
        const size_t q = (size_t)k * nc + j;
        double d = in ? (double)inv_dd[q] : 0.0;
        double a = in ? -(double)up[q] * d : 1.0;
        double b = in ? ys[c] * d : 0.0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double an = __shfl_down(a, off, 64), bn = __shfl_down(b, off, 64);
            if (lane + off < 64) {
                b = a * bn + b;
                a = a * an;
            }
        }
        const double xv = a * carry + b;
        if (in) x[q] = (T)xv;
        carry = __shfl(xv, 0, 64);
    }
}

// rhs of the pseudo-Schur system: -rho (P d)^k, dsum[k] = 1^T d^k
template <typename T>
__global__ void k_schur_rhs(const double *__restrict__ ac, int nc, double area, const double *__restrict__ dsum,
                            const T *__restrict__ rhoT, const T *__restrict__ d, T *__restrict__ out) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (j >= nc) return;
    const size_t q = (size_t)k * nc + j;
    out[q] = (T)(-(double)rhoT[q] * ((double)d[q] - ac[j] * dsum[k] / area));
}

// y^k = M'^-1 A~^k z^k  (before P^T)
template <typename T>
__global__ void k_coarse_lap_scaled(MeshView m, const T *__restrict__ z, const T *__restrict__ wc,
                                    T *__restrict__ y) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (j >= m.nc) return;
    const T *zk = z + (size_t)k * m.nc;
    const T *wck = wc + (size_t)k * m.nce;
    const double zj = (double)zk[j];
    double at = 0.0;
    for (int t = 0; t < m.wcc; ++t) {
        const int e = m.cc_edge[t * m.nc + j];
        if (e < 0) break;
        at += (double)wck[e] * (zj - (double)zk[m.cc_nb[t * m.nc + j]]);
    }
    y[(size_t)k * m.nc + j] = (T)(at / m.ac[j]);
}

// b^k = c^k - (B^T y)^k (type T, y already projected)
template <typename T>
__global__ void k_bt_rhs(MeshView m, int K, double dt, const T *__restrict__ c, const T *__restrict__ y,
                         const T *__restrict__ g, T *__restrict__ b) {
    const int i = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (i >= m.nf) return;
    auto yat = [&](int l, int cc) -> double { return (l >= 0 && l < K) ? (double)y[(size_t)l * m.nc + cc] : 0.0; };
    double v = 0.0;
    for (int t = 0; t < m.wo; ++t) {
        const int cc = m.fo_c[t * m.nf + i];
        if (cc < 0) break;
        v += m.fo_w[t * m.nf + i] * (yat(k - 1, cc) - yat(k, cc)) / dt;
    }
    const T *gk = g + (size_t)k * m.ne;
    for (int t = 0; t < m.wf; ++t) {
        const int e = m.cf_edge[t * m.nf + i];
        if (e < 0) break;
        const double sgn = (m.eK[e] == i) ? 1.0 : -1.0;
        const int rK = m.erK[e], rL = m.erL[e];
        const double lam = m.elam[e];
        const double re = lam * (yat(k - 1, rK) + yat(k, rK)) + (1.0 - lam) * (yat(k - 1, rL) + yat(k, rL));
        v += 0.5 * sgn * m.elen[e] * (double)gk[e] * re;
    }
    const size_t q = (size_t)k * m.nf + i;
    b[q] = (T)((double)c[q] - v);
}

// ------------------------------------------------------------- multigrid
// Graph Laplacian of one level, all slices: (A x)_i = sum_t w_e (x_i - x_nb)
struct LevelView {
    int n, w, ne;
    const int *nb, *ed;
};

// Galerkin edge weights of the next level: wn[k][c] = sum over member edges
template <typename T>
__global__ void k_mg_coarse_w(int ne_next, int ne, const int *__restrict__ ptr, const int *__restrict__ idx,
                              const T *__restrict__ w, T *__restrict__ wn) {
    const int c = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (c >= ne_next) return;
    double v = 0.0;
    for (int p = ptr[c]; p < ptr[c + 1]; ++p) v += (double)w[(size_t)k * ne + idx[p]];
    wn[(size_t)k * ne_next + c] = (T)v;
}

template <typename T>
__global__ void k_mg_diag(LevelView L, const T *__restrict__ w, T *__restrict__ dinv) {
    const int i = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (i >= L.n) return;
    double d = 0.0;
    for (int t = 0; t < L.w; ++t) {
        const int e = L.ed[t * L.n + i];
        if (e < 0) break;
        d += (double)w[(size_t)k * L.ne + e];
    }
    dinv[(size_t)k * L.n + i] = (T)(d > 0.0 ? 1.0 / d : 0.0);
}

template <typename TW, typename TX>
__device__ __forceinline__ double lap_row(const LevelView &L, const TW *w, const TX *x, int i) {
    const double xi = (double)x[i];
    double v = 0.0;
    for (int t = 0; t < L.w; ++t) {
        const int e = L.ed[t * L.n + i];
        if (e < 0) break;
        v += (double)w[e] * (xi - (double)x[L.nb[t * L.n + i]]);
    }
    return v;
}

// y = A x on every slice; weights TW (FP32 in the mixed path), vectors TX
template <typename TW, typename TX>
__global__ void k_mg_apply(LevelView L, const TW *__restrict__ w, const TX *__restrict__ x, TX *__restrict__ y) {
    const int i = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (i >= L.n) return;
    y[(size_t)k * L.n + i] = (TX)lap_row(L, w + (size_t)k * L.ne, x + (size_t)k * L.n, i);
}

// Chebyshev smoothing of D^-1 A on [lo, hi] (Saad, Alg. 12.1):
// init: r = D^-1 (b - A x) (x = 0 when zero_x), d = r / theta
template <typename T>
__global__ void k_cheb_init(LevelView L, const T *__restrict__ w, const T *__restrict__ dinv,
                            const T *__restrict__ b, T *__restrict__ x, T *__restrict__ r, T *__restrict__ d,
                            double theta, int zero_x) {
    const int i = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (i >= L.n) return;
    const size_t q = (size_t)k * L.n + i;
    double ax = 0.0;
    if (zero_x) x[q] = (T)0;
    else ax = lap_row(L, w + (size_t)k * L.ne, x + (size_t)k * L.n, i);
    const double rr = ((double)b[q] - ax) * (double)dinv[q];
    r[q] = (T)rr;
    d[q] = (T)(rr / theta);
}

// step: x += d; r -= D^-1 A d; d' = c1 d + c2 r
// FINE tags the launches at the finest level, so that profilers list them
// as a kernel of their own (one launch shape)
template <typename T, int FINE = 0>
__global__ void k_cheb_step(LevelView L, const T *__restrict__ w, const T *__restrict__ dinv, T *__restrict__ x,
                            T *__restrict__ r, const T *__restrict__ d, T *__restrict__ dn, double c1, double c2) {
    const int i = xcd_band_block() * BS + threadIdx.x, k = blockIdx.y;
    if (i >= L.n) return;
    const size_t q = (size_t)k * L.n + i;
    const double ad = lap_row(L, w + (size_t)k * L.ne, d + (size_t)k * L.n, i);
    const double di = (double)d[q];
    x[q] = (T)((double)x[q] + di);
    const double rn = (double)r[q] - ad * (double)dinv[q];
    r[q] = (T)rn;
    dn[q] = (T)(c1 * di + c2 * rn);
}

// restriction of the residual: bc[c] = sum_{i in agg c} (b - A x)_i
template <typename T>
__global__ void k_mg_restrict(LevelView L, int n_next, const int *__restrict__ ptr, const int *__restrict__ idx,
                              const T *__restrict__ w, const T *__restrict__ b, const T *__restrict__ x,
                              T *__restrict__ bc) {
    const int c = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (c >= n_next) return;
    const T *wk = w + (size_t)k * L.ne;
    const T *xk = x + (size_t)k * L.n;
    const T *bk = b + (size_t)k * L.n;
    double v = 0.0;
    for (int p = ptr[c]; p < ptr[c + 1]; ++p) {
        const int i = idx[p];
        v += (double)bk[i] - lap_row(L, wk, xk, i);
    }
    bc[(size_t)k * n_next + c] = (T)v;
}

template <typename T>
__global__ void k_mg_prolong(int n, int n_next, const int *__restrict__ agg, const T *__restrict__ xc,
                             T *__restrict__ x, double alpha) {
    const int i = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (i >= n) return;
    const size_t q = (size_t)k * n + i;
    x[q] = (T)((double)x[q] + alpha * (double)xc[(size_t)k * n_next + agg[i]]);
}

// per-slice PCG updates with host-provided per-slice scalars in alpha/beta
template <typename T>
__global__ void k_pcg_xr(int n, const double *__restrict__ alpha, const T *__restrict__ p, const T *__restrict__ q,
                         T *__restrict__ x, T *__restrict__ r) {
    const int i = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (i >= n) return;
    const size_t o = (size_t)k * n + i;
    const double a = alpha[k];
    x[o] = (T)((double)x[o] + a * (double)p[o]);
    r[o] = (T)((double)r[o] - a * (double)q[o]);
}

template <typename T>
__global__ void k_pcg_p(int n, const double *__restrict__ beta, const T *__restrict__ z, T *__restrict__ p) {
    const int i = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (i >= n) return;
    const size_t o = (size_t)k * n + i;
    p[o] = (T)((double)z[o] + beta[k] * (double)p[o]);
}

// y = x * d (inv = 0) or y = x / d (inv = 1), d a per-entry FP64 scale
template <typename T>
__global__ void k_dscale(size_t n, const double *__restrict__ d, int inv, const T *__restrict__ x, T *__restrict__ y) {
    for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) {
        const double di = d[i];
        const double f = inv ? (di != 0.0 ? 1.0 / di : 1.0) : di;
        y[i] = (T)((double)x[i] * f);
    }
}

// ------------------------------------------- pseudo-Schur multigrid levels
// Level l >= 1 stores its Galerkin operator as v[((d * w + slot) * K + k) * n + a],
// d = time offset + 1 in {0, 1, 2}, slot over the ELL stencil nbr (slot 0 = self).
struct SLevelView {
    int n, w;
    const int *nbr;
};

// probe at level l-1 for the colours of level l: 1 at (k, j) with k % 3 == tc
// and the colour of j's aggregate equal to c
template <typename T>
__global__ void k_sprobe(int n_prev, const int *__restrict__ agg, const int *__restrict__ color, int tc, int c,
                         T *__restrict__ p) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (j < n_prev) p[(size_t)k * n_prev + j] = (T)((k % 3 == tc && color[agg[j]] == c) ? 1.0 : 0.0);
}

// R[k][a] = sum over the members j of aggregate a of r[k][j]
template <typename T>
__global__ void k_srestrict(int n_next, int n, const int *__restrict__ ptr, const int *__restrict__ idx,
                            const T *__restrict__ r, T *__restrict__ R) {
    const int a = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (a >= n_next) return;
    double v = 0.0;
    for (int p = ptr[a]; p < ptr[a + 1]; ++p) v += (double)r[(size_t)k * n + idx[p]];
    R[(size_t)k * n_next + a] = (T)v;
}

// scatter a restricted probe response into the stencil slot of the
// colour-c neighbour, at the single time offset whose level is in class tc
template <typename T>
__global__ void k_sscatter(SLevelView L, int K, const int *__restrict__ slot_of, int tc, int c,
                           const T *__restrict__ R, T *__restrict__ v) {
    const int a = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (a >= L.n) return;
    const int slot = slot_of[(size_t)c * L.n + a];
    if (slot < 0) return;
    for (int d = -1; d <= 1; ++d) {
        const int kk = k + d;
        if (kk < 0 || kk >= K || kk % 3 != tc) continue;
        v[(((size_t)(d + 1) * L.w + slot) * K + k) * L.n + a] = R[(size_t)k * L.n + a];
    }
}

// y = S x, or y = b - S x when b is given
template <typename T>
__global__ void k_sspmv(SLevelView L, int K, const T *__restrict__ v, const T *__restrict__ x,
                        const T *__restrict__ b, T *__restrict__ y) {
    const int a = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (a >= L.n) return;
    double acc = 0.0;
    for (int s = 0; s < L.w; ++s) {
        const int nb = L.nbr[(size_t)s * L.n + a];
        if (nb < 0) break;
        for (int d = -1; d <= 1; ++d) {
            const int kk = k + d;
            if (kk < 0 || kk >= K) continue;
            acc += (double)v[(((size_t)(d + 1) * L.w + s) * K + k) * L.n + a] * (double)x[(size_t)kk * L.n + nb];
        }
    }
    const size_t q = (size_t)k * L.n + a;
    y[q] = (T)(b ? (double)b[q] - acc : acc);
}

// time diagonals of a level's own stencil slot
template <typename T>
__global__ void k_sdiag(SLevelView L, int K, const T *__restrict__ v, double *__restrict__ d0,
                        double *__restrict__ dl, double *__restrict__ du) {
    const int a = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (a >= L.n) return;
    const size_t q = (size_t)k * L.n + a;
    dl[q] = (double)v[(((size_t)0 * L.w + 0) * K + k) * L.n + a];
    d0[q] = (double)v[(((size_t)1 * L.w + 0) * K + k) * L.n + a];
    du[q] = (double)v[(((size_t)2 * L.w + 0) * K + k) * L.n + a];
}

template <typename T>
__global__ void k_sprolong(int n, int n_next, const int *__restrict__ agg, const T *__restrict__ xc, double w,
                           T *__restrict__ x) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (j >= n) return;
    const size_t q = (size_t)k * n + j;
    x[q] = (T)((double)x[q] + w * (double)xc[(size_t)k * n_next + agg[j]]);
}

// ----------------------------------------------------- Newton step pieces
// Newton right-hand side of the projected system: f = -F_phi (copied),
// g~ = -F_rho + a' (F_s) / rho, written as (f; g~) in out; P applied later.
__global__ void k_newton_rhs(MeshView m, StateView S, const double *__restrict__ F, double *__restrict__ out,
                             double *__restrict__ gt, double *__restrict__ part, size_t nphi, size_t mrho) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    double v = 0.0;
    if (j < m.nc) {
        const size_t q = (size_t)k * m.nc + j;
        const double g = -F[nphi + q], h = -F[nphi + mrho + q];
        v = g - m.ac[j] * h / S.rho[q];
        gt[q] = v;
        out[nphi + q] = v;
    }
    v = block_sum(v);
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = v;
}

__global__ void k_neg_copy(size_t n, const double *__restrict__ x, double *__restrict__ y) {
    for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) y[i] = -x[i];
}

// recovery residual r = g~ - B dphi_bar + C drho (B dphi_bar in bphi), partial slice sums
__global__ void k_recover_r(int nc, const double *__restrict__ ac, const double *__restrict__ gt,
                            const double *__restrict__ bphi, const double *__restrict__ drho, StateView S,
                            double *__restrict__ part) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    double v = 0.0;
    if (j < nc) {
        const size_t q = (size_t)k * nc + j;
        v = gt[q] - bphi[q] + ac[j] * S.s[q] / S.rho[q] * drho[q];
    }
    v = block_sum(v);
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = v;
}

// dphi^k += shift[k]
__global__ void k_add_shift(int nf, const double *__restrict__ shift, double *__restrict__ dphi) {
    const int i = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (i < nf) dphi[(size_t)k * nf + i] += shift[k];
}

// ds = (h - s drho)/rho with h = -(rho s - mu); partial min of the step ratios
// ds = (h - s drho) / rho and the largest steps keeping rho (part[b]) and
// s (part[nblk + b]) positive, per block
__global__ void k_ds_ratio(size_t n, StateView S, double mu, const double *__restrict__ drho,
                           double *__restrict__ ds, double *__restrict__ part) {
    double ap = DBL_MAX, ad = DBL_MAX;
    for (size_t q = (size_t)blockIdx.x * BS + threadIdx.x; q < n; q += (size_t)gridDim.x * BS) {
        const double r = S.rho[q], s = S.s[q], dr = drho[q];
        const double h = -(r * s - mu);
        const double d = (h - s * dr) / r;
        ds[q] = d;
        if (dr < 0) ap = fmin(ap, -r / dr);
        if (d < 0) ad = fmin(ad, -s / d);
    }
    ap = block_min(ap);
    ad = block_min(ad);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = ap;
        part[gridDim.x + blockIdx.x] = ad;
    }
}

// Diagonal of the K+1 weighted Laplacians A^k (FP64): d^k_i = sum over the
// edges of cell i of tw_e rho~^k_e (the SIMPLE approximation Diag(A)).
__global__ void k_lap_diag(MeshView m, StateView S, double *__restrict__ d) {
    const int i = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (i >= m.nf) return;
    double v = 0.0;
    for (int t = 0; t < m.wf; ++t) {
        const int e = m.cf_edge[t * m.nf + i];
        if (e < 0) break;
        v += m.etw[e] * rho_edge(m, S, k, e);
    }
    d[(size_t)k * m.nf + i] = v;
}

// Largest step t in [0, amax] that keeps every cell in the neighbourhood
// (rho + t drho)(s + t ds) >= gmu of the central path; per-block minima.
// Per cell q(t) = a t^2 + b t + c with a = drho ds, b = rho ds + s drho,
// c = rho s - gmu > 0, and the bound is its first positive root; cells
// already outside the neighbourhood (c <= 0) do not constrain the step.
__global__ void k_central_alpha(size_t n, StateView S, const double *__restrict__ drho,
                                const double *__restrict__ ds, double gmu, double amax,
                                double *__restrict__ part) {
    double am = amax;
    for (size_t q = (size_t)blockIdx.x * BS + threadIdx.x; q < n; q += (size_t)gridDim.x * BS) {
        const double r = S.rho[q], s = S.s[q], dr = drho[q], d = ds[q];
        const double c = r * s - gmu;
        if (!(c > 0.0)) continue;
        const double a = dr * d, b = r * d + s * dr;
        double t = DBL_MAX;
        if (a == 0.0) {
            if (b < 0.0) t = -c / b;
        } else {
            const double disc = b * b - 4.0 * a * c;
            if (disc >= 0.0) {
                const double sq = sqrt(disc);
                const double qq = -0.5 * (b + (b >= 0.0 ? sq : -sq));   // stable pair of roots
                const double t1 = qq / a, t2 = c / qq;
                if (t1 > 0.0) t = fmin(t, t1);
                if (t2 > 0.0) t = fmin(t, t2);
            }
        }
        am = fmin(am, t);
    }
    am = block_min(am);
    if (threadIdx.x == 0) part[blockIdx.x] = am;
}

// x += alpha dx
__global__ void k_axpy(size_t n, double a, const double *__restrict__ dx, double *__restrict__ x) {
    for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += (size_t)gridDim.x * BS) x[i] += a * dx[i];
}

// rho^k *= m0 / mass[k]
__global__ void k_renorm(int nc, const double *__restrict__ mass, double m0, double *__restrict__ rho) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    if (j < nc) rho[(size_t)k * nc + j] *= m0 / mass[k];
}

// ------------------------------------------------------------- outputs
// partial sums of W rho~ g^2 over edges and potential levels
__global__ void k_ke_partial(MeshView m, StateView S, double *__restrict__ part) {
    const int e = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    double v = 0.0;
    if (e < m.ne) {
        const double g = grad_phi(m, S.phi + (size_t)k * m.nf, e);
        v = m.eW[e] * rho_edge(m, S, k, e) * g * g;
    }
    v = block_sum(v);
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = v;
}

// envelope parts per coarse cell: R_T (g^2) at the first and last potential
// levels and Omega^T phi there.  Writes 4 arrays of nc.
__global__ void k_boundary_terms(MeshView m, StateView S, const double *__restrict__ phi_first,
                                 const double *__restrict__ phi_last, double *__restrict__ om_first,
                                 double *__restrict__ om_last, double *__restrict__ rt_first,
                                 double *__restrict__ rt_last) {
    const int j = blockIdx.x * BS + threadIdx.x;
    if (j >= m.nc) return;
    double o1 = 0.0, o2 = 0.0, r1 = 0.0, r2 = 0.0;
    for (int t = 0; t < m.woc; ++t) {
        const int f = m.co_f[t * m.nc + j];
        if (f < 0) break;
        o1 += m.co_w[t * m.nc + j] * phi_first[f];
        o2 += m.co_w[t * m.nc + j] * phi_last[f];
    }
    for (int t = 0; t < m.wr; ++t) {
        const int e = m.cr_e[t * m.nc + j];
        if (e < 0) break;
        const double g1 = grad_phi(m, phi_first, e), g2 = grad_phi(m, phi_last, e);
        r1 += m.cr_w[t * m.nc + j] * g1 * g1;
        r2 += m.cr_w[t * m.nc + j] * g2 * g2;
    }
    om_first[j] = o1; om_last[j] = o2; rt_first[j] = r1; rt_last[j] = r2;
}

// adjoint corrections: out[j] = sgn_t Omega^T q / dt + 1/2 R_T(g * grad q) at one level
__global__ void k_adjoint_corr(MeshView m, const double *__restrict__ ph, const double *__restrict__ q,
                               double tsign, double dt, double *__restrict__ out) {
    const int j = blockIdx.x * BS + threadIdx.x;
    if (j >= m.nc) return;
    double v = 0.0;
    for (int t = 0; t < m.woc; ++t) {
        const int f = m.co_f[t * m.nc + j];
        if (f < 0) break;
        v += tsign * m.co_w[t * m.nc + j] * q[f] / dt;
    }
    double gg = 0.0;
    for (int t = 0; t < m.wr; ++t) {
        const int e = m.cr_e[t * m.nc + j];
        if (e < 0) break;
        gg += m.cr_w[t * m.nc + j] * grad_phi(m, ph, e) * grad_phi(m, q, e);
    }
    out[j] = v + 0.5 * gg;
}

// Adjoint right-hand side of the cost gradient: the rho block of the Newton
// system gets dt a' s (phi block zero, set by the caller); gt holds the same
// values for the recovery.  Partial sums of squares for its norm.
__global__ void k_grad_rhs(int nc, const double *__restrict__ ac, StateView S, double *__restrict__ gt,
                           double *__restrict__ out_rho, double *__restrict__ part) {
    const int j = blockIdx.x * BS + threadIdx.x, k = blockIdx.y;
    double sq = 0.0;
    if (j < nc) {
        const size_t q = (size_t)k * nc + j;
        const double v = S.dt * ac[j] * S.s[q];
        gt[q] = v;
        out_rho[q] = v;
        sq = v * v;
    }
    sq = block_sum(sq);
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = sq;
}

// Gradient assembly per coarse cell from the envelope parts (Omega^T phi and
// R_T (grad phi)^2 at the first / last potential level) and the adjoint
// corrections:
//   g_in = -Omega^T phi^1 - dt/4 R_T (grad phi^1)^2 - corr_first
//   g_f  =  Omega^T phi^{K+1} - dt/4 R_T (grad phi^{K+1})^2 - corr_last
// b holds [corr_first, corr_last, om_first, om_last, rt_first, rt_last],
// nc each.  Partial sums of a' g_in, a' g_f and a' a' per block
// (part[0 / 1 / 2 * nblk + b]) for the projection orthogonal to a'.
__global__ void k_grad_assemble(int nc, const double *__restrict__ ac, double dt, const double *__restrict__ b,
                                double *__restrict__ gi, double *__restrict__ gf, double *__restrict__ part) {
    const int j = blockIdx.x * BS + threadIdx.x;
    double si = 0.0, sf = 0.0, sa = 0.0;
    if (j < nc) {
        const double vi = -b[2 * (size_t)nc + j] - 0.25 * dt * b[4 * (size_t)nc + j] - b[j];
        const double vf = b[3 * (size_t)nc + j] - 0.25 * dt * b[5 * (size_t)nc + j] - b[(size_t)nc + j];
        gi[j] = vi;
        gf[j] = vf;
        si = ac[j] * vi;
        sf = ac[j] * vf;
        sa = ac[j] * ac[j];
    }
    si = block_sum(si);
    sf = block_sum(sf);
    sa = block_sum(sa);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = si;
        part[gridDim.x + blockIdx.x] = sf;
        part[2 * gridDim.x + blockIdx.x] = sa;
    }
}

// g -= a' (a'^T g) / (a'^T a') for both gradients; sums = [a'g_in, a'g_f, a'a']
__global__ void k_grad_project(int nc, const double *__restrict__ ac, const double *__restrict__ sums,
                               double *__restrict__ gi, double *__restrict__ gf) {
    const int j = blockIdx.x * BS + threadIdx.x;
    if (j >= nc) return;
    const double aa = sums[2];
    gi[j] -= ac[j] * sums[0] / aa;
    gf[j] -= ac[j] * sums[1] / aa;
}

}  // namespace kern
}  // namespace otbb
