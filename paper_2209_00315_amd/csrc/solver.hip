// Interior-point solver: state, operators, BB preconditioner, FGMRES,
// Newton step, continuation, outputs, gradient, and the C ABI.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <thread>
#include <tuple>
#include <type_traits>
#include <atomic>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "kprof.hpp"
#include "mesh.hpp"

using namespace otbb;
using namespace otbb::kern;

namespace otbb {

namespace kprof {
Prof &prof() {
    static Prof p;
    return p;
}
// synchronise with every pending pair and add its time (caller holds mu)
void drain(Prof &P) {
    for (size_t i = 0; i < P.used; ++i) {
        OT_HIP(hipEventSynchronize(P.pool[i].second));
        float t = 0.0f;
        OT_HIP(hipEventElapsedTime(&t, P.pool[i].first, P.pool[i].second));
        P.ms += t;
        P.bytes += P.pend[i];
        P.launches++;
    }
    P.used = 0;
}
Ev take_slot(double bytes) {
    Prof &P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    if (P.used == P.pool.size()) {
        if (P.pool.size() < 4096) {
            std::pair<hipEvent_t, hipEvent_t> e;
            OT_HIP(hipEventCreate(&e.first));
            OT_HIP(hipEventCreate(&e.second));
            P.pool.push_back(e);
            P.pend.push_back(0.0);
        } else {
            drain(P);
        }
    }
    Ev e;
    e.a = P.pool[P.used].first;
    e.b = P.pool[P.used].second;
    P.pend[P.used] = bytes;
    P.used++;
    return e;
}
}  // namespace kprof

// Largest Krylov basis any option combination can request (restart and
// inner_restart are validated against it); sizes every Krylov scratch.
constexpr int kMaxBasis = 401;
constexpr int kMultidotBlocks = 512;
constexpr int kUpdateBlocks = 8192;
// time levels per thread of the two time-blocked pseudo-Schur passes
// (M^-1 B~ z, output) for FP32 [0] and FP64 [1] operands; 0 selects the
// one-level-per-thread kernels.  Measured at 256^2, K = 64: blocking by 16
// cuts the FP32 M^-1 B~ z pass from 72 to 28 us and the FP64 passes from
// 83 / 103 to 53 / 65 us, while the FP32 output pass is fastest unblocked
// (76 us; blocked 92-128 us, fewer independent gathers in flight).
// These are the defaults; each BB preconditioner measures the candidates on
// its own mesh and K at its first linearisation (autotune_schur_blocking)
// unless otbb_debug_set_schur_blocking has fixed them.
static int g_schur_tb[2][2] = {{16, 0}, {16, 16}};
static bool g_schur_tb_fixed[2] = {false, false};
// Autotuned choices, shared by every preconditioner of the same shape in
// the process: the blocked and per-level passes round differently, so a
// choice that depended on each state's own timing (which concurrent
// streams perturb) would make results depend on scheduling.  Key: n_f,
// n_c, fine edges, K, FP64 or not.
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int, int>, std::pair<int, int>> g_tune_cache;
// pseudo-Schur V-cycle parameters of BB preconditioners created afterwards
// (otbb_debug_set_schur_mg)
struct SchurMGParams {
    double omega = 0.5;          // damping of the time-line Jacobi smoother
    int nu = 2;                  // pre- and post-smoothing steps
    int coarse_its = 6;          // smoothing steps on the coarsest level
    double alpha = 1.0;          // scale of the prolongated coarse correction
};
static SchurMGParams g_smg;
// longest time line the wavefront-scan tridiagonal solve handles
constexpr int kTriScanMaxK = 64 * kern::kTriScanChunks;

static thread_local std::string g_last_error = "no error";
void set_last_error(const std::string &msg) { g_last_error = msg; }

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

static inline dim3 grid2(int n, int nseg) { return dim3((unsigned)std::max(1, ceil_div(n, BS)), (unsigned)nseg); }
static inline int grid1(size_t n, int cap = 1024) {
    return (int)std::max<size_t>(1, std::min<size_t>((n + BS - 1) / BS, (size_t)cap));
}

MeshView mesh_view(const ot_mesh *m) {
    const MeshHost &h = m->h;
    MeshView v;
    v.nf = h.nf; v.nc = h.nc; v.ne = h.ne; v.nce = h.nce;
    v.wf = h.wf; v.wo = h.wo; v.woc = h.woc; v.wr = h.wr; v.wcc = h.wcc;
    v.a = m->a; v.ac = m->ac; v.elam = m->elam; v.etw = m->etw; v.eW = m->eW; v.einvd = m->einvd;
    v.elen = m->elen; v.cetw = m->cetw; v.celam = m->celam; v.fo_w = m->fo_w; v.co_w = m->co_w; v.cr_w = m->cr_w;
    v.eK = m->eK; v.eL = m->eL; v.erK = m->erK; v.erL = m->erL; v.ceI = m->ceI; v.ceJ = m->ceJ;
    v.cf_edge = m->cf_edge; v.cf_nb = m->cf_nb; v.fo_c = m->fo_c; v.co_f = m->co_f; v.cr_e = m->cr_e;
    v.cc_edge = m->cc_edge; v.cc_nb = m->cc_nb;
    v.cr_k = m->cr_k; v.cr_l = m->cr_l; v.cr_g = m->cr_g; v.cr_g2 = m->cr_g2;
    v.cf_rk = m->cf_rk; v.cf_rl = m->cf_rl; v.cf_lam = m->cf_lam; v.cf_bw = m->cf_bw; v.cf_tw = m->cf_tw;
    return v;
}

// ---------------------------------------------------------------------------
// Reduction scratch bound to a stream
// ---------------------------------------------------------------------------
struct Reducer {
    hipStream_t s = nullptr;
    DBuf<double> part, dev;
    double *host = nullptr;      // pinned
    size_t host_n = 0;
    void init(size_t npart, size_t ndev, hipStream_t st) {
        s = st;
        part.alloc(npart);
        dev.alloc(ndev);
        host_n = ndev;
        OT_HIP(hipHostMalloc((void **)&host, ndev * sizeof(double), hipHostMallocDefault));
    }
    ~Reducer() { if (host) (void)hipHostFree(host); }
    // copy n device scalars to host and wait
    const double *fetch(const double *d, size_t n) {
        OT_REQUIRE(n <= host_n, OT_EINVAL, "internal: reduction fetch too large");
        OT_HIP(hipGetLastError());
        OT_HIP(hipMemcpyAsync(host, d, n * sizeof(double), hipMemcpyDeviceToHost, s));
        OT_HIP(hipStreamSynchronize(s));
        return host;
    }
    // final reduction of nseg segments of nblk partials into dev[off..]
    double *seg_final(int nseg, int nblk, size_t off = 0) {
        k_seg_final<<<nseg, BS, 0, s>>>(part, nblk, dev.p + off);
        return dev.p + off;
    }
};

}  // namespace otbb

// ---------------------------------------------------------------------------
// State
// ---------------------------------------------------------------------------
struct PrecBase {
    virtual ~PrecBase() = default;
    virtual void setup(ot_state *st) = 0;
    virtual void apply(ot_state *st, const double *r, double *z) = 0;
    // component access for the inspection entry points (FP64 device in/out)
    virtual void schur_apply_d(ot_state *st, const double *z, double *out) = 0;
    virtual int schur_solve_d(ot_state *st, const double *rhs, double *z, double tol, int maxit) = 0;
    virtual void tri_diagonals_d(ot_state *st, double *d0, double *dl, double *du) = 0;
    virtual void tri_solve_d(ot_state *st, const double *r, double *x) = 0;
    virtual int laplace_solve_d(ot_state *st, const double *b, double *x, double tol, int maxit) = 0;
    virtual void vcycle_d(ot_state *st, const double *b, double *x) = 0;
    virtual size_t level_data_d(ot_state *st, int level, int what, double *out) = 0;
};

struct ot_state {
    const ot_mesh *mesh = nullptr;
    int K = 0;
    ot_options opt;
    hipStream_t stream = nullptr;
    size_t nphi = 0, mrho = 0, N = 0;
    double mu = 1.0, m0 = 0.0, dt = 0.0, area = 0.0;
    DBuf<double> phi, rho, s, rin, rf;
    DBuf<double> F, rhs, sol, gt, tmpN, tmpr, ds, sums, shift;
    DBuf<double> V, Z;
    Reducer red;
    // preconditioners built so far, by kind (2 * preconditioner + precision),
    // kept for retries and switches; prec points at the active one
    std::map<int, std::unique_ptr<PrecBase>> precs;
    PrecBase *prec = nullptr;
    int prec_kind = -1;
    bool hybrid_simple = false;                // OT_PREC_HYBRID has switched to SIMPLE
    bool lin_valid = false;
    ot_stats acc{};
    // last FGMRES info
    int last_iters = 0;
    double last_relres = 0.0;
    bool last_converged = false;
    bool no_plateau = false;                   // FGMRES runs to its cap (the retry of a failed solve)

    StateView view() const {
        StateView v;
        v.K = K; v.dt = dt; v.area = area;
        v.phi = phi; v.rho = rho; v.s = s; v.rin = rin; v.rf = rf;
        return v;
    }
};

namespace otbb {

// slice sums sums[k] = sum_i w_i x[k n + i] on device (nseg slices)
template <typename T>
static double *slice_sums(ot_state *st, const T *x, const double *w, int n, int nseg, double *out) {
    int nblk = std::min(256, std::max(1, ceil_div(n, BS)));
    k_seg_partial<T><<<dim3(nblk, nseg), BS, 0, st->stream>>>(x, w, n, st->red.part);
    k_seg_final<<<nseg, BS, 0, st->stream>>>(st->red.part, nblk, out);
    return out;
}

template <typename T>
static double *slice_dots(ot_state *st, const T *x, const T *y, int n, int nseg, double *out) {
    int nblk = std::min(256, std::max(1, ceil_div(n, BS)));
    k_seg_dot_partial<T><<<dim3(nblk, nseg), BS, 0, st->stream>>>(x, y, n, st->red.part);
    k_seg_final<<<nseg, BS, 0, st->stream>>>(st->red.part, nblk, out);
    return out;
}

template <typename T>
static double norm2(ot_state *st, const T *x, size_t n) {
    int nblk = grid1(n);
    k_nrm2_partial<T><<<nblk, BS, 0, st->stream>>>(n, x, st->red.part);
    double *d = st->red.seg_final(1, nblk);
    return std::sqrt(st->red.fetch(d, 1)[0]);
}

// ---------------------------------------------------------------------------
// Residual and saddle operator (FP64)
// ---------------------------------------------------------------------------
static double residual(ot_state *st) {
    const ot_mesh *m = st->mesh;
    MeshView mv = mesh_view(m);
    StateView sv = st->view();
    dim3 gf = grid2(m->h.nf, st->K + 1), gc = grid2(m->h.nc, st->K);
    k_res_phi<<<gf, BS, 0, st->stream>>>(mv, sv, st->F, st->red.part);
    int n1 = gf.x * gf.y;
    k_res_rho<<<gc, BS, 0, st->stream>>>(mv, sv, st->mu, st->F.p + st->nphi, st->F.p + st->nphi + st->mrho,
                                         st->red.part.p + n1);
    int n2 = gc.x * gc.y;
    double *d = st->red.seg_final(1, n1 + n2);
    return std::sqrt(st->red.fetch(d, 1)[0]);
}

// Scratch of y = J_P x: two slice-sum vectors (K each) and the per-block
// partial sums of the larger of its two reductions.
static size_t saddle_scratch_doubles(const ot_state *st) {
    const size_t K = st->K, nc = st->mesh->h.nc;
    const size_t nblk = std::max<size_t>(std::min<size_t>(256, (nc + BS - 1) / BS), (nc + BS - 1) / BS);
    return 2 * (K + 2) + nblk * K;
}

// y = J_P x (both length N, device), with caller-provided scratch: sums
// (2 (K + 2) doubles) and part (block partials), on stream s
static void apply_saddle_core(const ot_state *st, const double *x, double *y, double *sums, double *part,
                              hipStream_t s) {
    const ot_mesh *m = st->mesh;
    MeshView mv = mesh_view(m);
    StateView sv = st->view();
    const int K = st->K, nf = m->h.nf, nc = m->h.nc;
    double *cs = sums;                       // a'^T x_rho^k
    double *us = sums + K + 2;               // 1^T u^k
    {
        const int nblk = std::min(256, std::max(1, ceil_div(nc, BS)));
        k_seg_partial<double><<<dim3(nblk, K), BS, 0, s>>>(x + st->nphi, m->ac, nc, part);
        k_seg_final<<<K, BS, 0, s>>>(part, nblk, cs);
    }
    {
        // x, phi, y over the potential block; x_rho and rho once; geometry once
        const MeshHost &h = m->h;
        const double bytes = 8.0 * (3.0 * st->nphi + 2.0 * st->mrho) + 8.0 * h.wf * nf + 12.0 * h.wo * nf +
                             40.0 * h.ne;
        const kprof::Ev ev = kprof::take(OT_KPROF_SADDLE_PHI, 8, bytes);
        hipExtLaunchKernelGGL(k_saddle_phi, grid2(nf, K + 1), dim3(BS), 0, s, ev.a, ev.b, 0, mv, sv, x,
                              x + st->nphi, (const double *)cs, (const double *)nullptr, y);
    }
    dim3 gc = grid2(nc, K);
    k_opB<<<gc, BS, 0, s>>>(mv, sv, x, x + st->nphi, cs, 1.0, y + st->nphi, part);
    k_seg_final<<<K, BS, 0, s>>>(part, gc.x, us);
    k_proj_fix<double><<<gc, BS, 0, s>>>(m->ac, nc, us, st->area, y + st->nphi);
}

static void apply_saddle(ot_state *st, const double *x, double *y) {
    apply_saddle_core(st, x, y, st->sums.p, st->red.part.p, st->stream);
}

// ---------------------------------------------------------------------------
// Library-held scratch for the entry point that allocates nothing
// (ot_apply_saddle_noalloc).  One copy per device, held until the process
// ends; its device address is looked up once per device with that device
// current (the array's name is only a host-side handle).
// ---------------------------------------------------------------------------
constexpr size_t kNoallocScratch = 131072;            // doubles (1 MiB)
static __device__ __align__(256) double scratch[kNoallocScratch];
constexpr int kMaxDevices = 64;
static double *g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

// device address of `scratch` on the current device (looked up on first use)
static double *scratch_on_current_device() {
    int dev = -1;
    OT_HIP(hipGetDevice(&dev));
    OT_REQUIRE(dev >= 0 && dev < kMaxDevices, OT_EDEVICE, "device ordinal out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        OT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        OT_REQUIRE(p != nullptr, OT_EDEVICE, "no device address for the scratch array");
        g_scratch_dev[dev] = (double *)p;
    }
    return g_scratch_dev[dev];
}

// ---------------------------------------------------------------------------
// Krylov helpers
// ---------------------------------------------------------------------------
// Classical Gram-Schmidt with one reorthogonalisation of w against the nv
// vectors of V (leading dimension ld).  h[0..nv) receives the coefficients,
// the return value is |w| after orthogonalisation.  One host sync.
template <typename T>
static double cgs2(ot_state *st, const T *V, size_t ld, int nv, T *w, size_t n, double *h) {
    Reducer &R = st->red;
    OT_REQUIRE(nv >= 1 && nv <= kMaxBasis, OT_EINVAL, "internal: Krylov basis too large");
    const int nblk = grid1(n, kMultidotBlocks);
    const int nblk_u = grid1(n, kUpdateBlocks);
    const int ng = (nv + 7) / 8;
    OT_REQUIRE(R.part.n >= std::max((size_t)nv * nblk, (size_t)nblk_u) && R.dev.n >= 2 * (size_t)kMaxBasis + 1,
               OT_EINVAL, "internal: reduction scratch too small");
    double *h1 = R.dev.p, *h2 = R.dev.p + kMaxBasis, *nr = R.dev.p + 2 * kMaxBasis;
    for (int pass = 0; pass < 2; ++pass) {
        double *hp = pass ? h2 : h1;
        {
            const kprof::Ev ev = kprof::take(OT_KPROF_MULTIDOT, sizeof(T), (double)sizeof(T) * (nv + 1.0) * n);
            hipExtLaunchKernelGGL(k_multidot<T>, dim3(nblk, ng), dim3(BS), 0, st->stream, ev.a, ev.b, 0, n, V, ld,
                                  nv, (const T *)w, R.part.p);
        }
        k_seg_final<<<nv, BS, 0, st->stream>>>(R.part, nblk, hp);
        // the update walks all nv vectors per element: give it the whole
        // vector length in blocks so that every CU keeps loads in flight
        k_gs_update<T><<<nblk_u, BS, 0, st->stream>>>(n, V, ld, nv, hp, w, R.part);
    }
    k_seg_final<<<1, BS, 0, st->stream>>>(R.part, nblk_u, nr);
    const double *hh = R.fetch(R.dev.p, 2 * kMaxBasis + 1);
    for (int i = 0; i < nv; ++i) h[i] = hh[i] + hh[kMaxBasis + i];
    return std::sqrt(std::max(hh[2 * kMaxBasis], 0.0));
}

// Givens-rotation least squares state for (F)GMRES
struct Givens {
    int m;
    std::vector<double> H, cs, sn, g;
    explicit Givens(int m_) : m(m_), H((size_t)(m_ + 1) * m_, 0.0), cs(m_), sn(m_), g(m_ + 1, 0.0) {}
    double &h(int i, int j) { return H[(size_t)j * (m + 1) + i]; }
    void reset(double beta) { std::fill(g.begin(), g.end(), 0.0); g[0] = beta; }
    // column j holds h(0..j+1, j); returns |residual|
    double push(int j) {
        for (int i = 0; i < j; ++i) {
            double a = h(i, j), b = h(i + 1, j);
            h(i, j) = cs[i] * a + sn[i] * b;
            h(i + 1, j) = -sn[i] * a + cs[i] * b;
        }
        double a = h(j, j), b = h(j + 1, j);
        double r = std::hypot(a, b);
        cs[j] = r > 0 ? a / r : 1.0;
        sn[j] = r > 0 ? b / r : 0.0;
        h(j, j) = r;
        h(j + 1, j) = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        return std::fabs(g[j + 1]);
    }
    std::vector<double> solve(int k) {      // k columns
        std::vector<double> y(k, 0.0);
        for (int i = k - 1; i >= 0; --i) {
            double v = g[i];
            for (int q = i + 1; q < k; ++q) v -= h(i, q) * y[q];
            y[i] = h(i, i) != 0.0 ? v / h(i, i) : 0.0;
        }
        return y;
    }
};

}  // namespace otbb

// ---------------------------------------------------------------------------
// BB preconditioner, templated on the arithmetic type of its kernels
// ---------------------------------------------------------------------------
template <typename T>
struct BBPrec : PrecBase {
    int nf = 0, nc = 0, ne = 0, nce = 0, K = 0, nlev = 0;
    size_t nphi = 0, mrho = 0;
    DBuf<T> g, wc, rhoT, sT;
    std::vector<DBuf<T>> lw, ldinv;            // per level edge weights / inverse diagonal
    std::vector<DBuf<T>> lb, lx, lr, ld, ld2;  // per level work (level >= 1 use lb/lx)
    DBuf<double> d0, dl, du;
    DBuf<T> inv_dd, lm, up;
    DBuf<T> cT, dT, rhsS, zS, yT, bT, uT, vT, tmpm, tmpm2, tmpm3, probe;
    DBuf<double> VS, rhsc;                     // inner GMRES basis, scaled rhs (FP64 in both paths)
    // PCG work: the Krylov vectors and the operator are FP64 in both paths;
    // only the V-cycle (vb -> vx) runs in T.  An all-FP32 PCG stalls above
    // the 1e-6 relative residual the outer FGMRES needs at small mu.
    DBuf<double> px, pr, pz, pp, pq;
    DBuf<T> vb, vx;
    DBuf<double> coef;                         // per-slice alpha / beta
    // pseudo-Schur multigrid: per level >= 1 the Galerkin operator and its
    // time-line factors; per level work vectors (level 0 uses mrho sizes)
    int nsl = 0;
    std::vector<DBuf<T>> sv, sinv, slm, sup, sb, sx, sr, stt;
    DBuf<double> sd0, sdl, sdu;                // coarse-level diagonal scratch
    double somega = 0.5, s_alpha = 1.0;         // smoother damping, coarse-correction scale
    int s_nu = 2, s_coarse_its = 6;
    int mS = 20;
    int tb_b = -1, tb_o = -1;                  // pseudo-Schur pass blocking (autotuned)
    const double hi = 2.0, lo_ratio = 0.3, coarse_lo_ratio = 0.02;
    int nu = 2, coarse_deg = 8;
    // Over-correction of the piecewise-constant coarse-grid correction: plain
    // aggregation underestimates the smooth error; scaling by 1.8 keeps the
    // V-cycle symmetric and cuts PCG iterations from ~30 to ~7 on 256^2.
    double mg_alpha = 1.8;

    void alloc(ot_state *st) {
        const ot_mesh *m = st->mesh;
        nf = m->h.nf; nc = m->h.nc; ne = m->h.ne; nce = m->h.nce; K = st->K;
        nphi = st->nphi; mrho = st->mrho;
        nlev = (int)m->lv.size();
        mS = std::max(2, st->opt.inner_restart);
        somega = g_smg.omega; s_nu = g_smg.nu; s_coarse_its = g_smg.coarse_its; s_alpha = g_smg.alpha;
        g.alloc((size_t)(K + 1) * std::max(ne, 1));
        wc.alloc((size_t)K * std::max(nce, 1));
        rhoT.alloc(mrho); sT.alloc(mrho);
        lw.clear(); ldinv.clear(); lb.clear(); lx.clear(); lr.clear(); ld.clear(); ld2.clear();
        for (int l = 0; l < nlev; ++l) {
            const MGLevelDev &L = m->lv[l];
            lw.emplace_back((size_t)(K + 1) * std::max(L.ne, 1));
            ldinv.emplace_back((size_t)(K + 1) * L.n);
            lb.emplace_back((size_t)(K + 1) * L.n);
            lx.emplace_back((size_t)(K + 1) * L.n);
            lr.emplace_back((size_t)(K + 1) * L.n);
            ld.emplace_back((size_t)(K + 1) * L.n);
            ld2.emplace_back((size_t)(K + 1) * L.n);
        }
        d0.alloc(mrho); dl.alloc(mrho); du.alloc(mrho);
        inv_dd.alloc(mrho); lm.alloc(mrho); up.alloc(mrho);
        cT.alloc(nphi); dT.alloc(mrho); rhsS.alloc(mrho); zS.alloc(mrho); yT.alloc(mrho);
        bT.alloc(nphi); uT.alloc(nphi); vT.alloc(nphi); tmpm.alloc(mrho); tmpm2.alloc(mrho); tmpm3.alloc(mrho); probe.alloc(mrho);
        VS.alloc((size_t)(mS + 1) * mrho);
        rhsc.alloc(mrho);
        px.alloc(nphi); pr.alloc(nphi); pz.alloc(nphi); pp.alloc(nphi); pq.alloc(nphi);
        vb.alloc(nphi); vx.alloc(nphi);
        coef.alloc(2 * (K + 2));
        nsl = (int)m->slv.size();
        sv.clear(); sinv.clear(); slm.clear(); sup.clear(); sb.clear(); sx.clear(); sr.clear(); stt.clear();
        for (int l = 0; l < nsl; ++l) {
            const SLevelDev &L = m->slv[l];
            const size_t nk = (size_t)K * L.n;
            sv.emplace_back(l == 0 ? (size_t)1 : 3 * (size_t)L.w * nk);
            sinv.emplace_back(l == 0 ? (size_t)1 : nk);
            slm.emplace_back(l == 0 ? (size_t)1 : nk);
            sup.emplace_back(l == 0 ? (size_t)1 : nk);
            sb.emplace_back(nk); sx.emplace_back(nk); sr.emplace_back(nk); stt.emplace_back(nk);
        }
        const size_t n1 = nsl > 1 ? (size_t)K * m->slv[1].n : 1;
        sd0.alloc(n1); sdl.alloc(n1); sdu.alloc(n1);
    }

    SLevelView slview(const ot_mesh *m, int l) const {
        SLevelView v;
        v.n = m->slv[l].n; v.w = m->slv[l].w; v.nbr = m->slv[l].nbr;
        return v;
    }

    // S_l x (level 0: the matrix-free pseudo-Schur operator); b != null: b - S_l x
    void s_apply(ot_state *st, int l, const T *x, const T *b, T *y) {
        const ot_mesh *m = st->mesh;
        if (l == 0) {
            schur_apply(st, x, y);
            if (b) k_axpby<T><<<grid1(mrho), BS, 0, st->stream>>>(mrho, 1.0, b, -1.0, y);
            return;
        }
        k_sspmv<T><<<grid2(m->slv[l].n, K), BS, 0, st->stream>>>(slview(m, l), K, sv[l], x, b, y);
    }

    void s_tri(ot_state *st, int l, const T *r, T *x) {
        const int n = st->mesh->slv[l].n;
        if (l == 0) tri_apply(st, r, x);
        else tri_launch<0>(st->stream, n, sinv[l], slm[l], sup[l], r, x, kprof::Ev{});
    }

    // assemble the Galerkin operators of levels >= 1 by probing the level above
    void s_setup(ot_state *st) {
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        for (int l = 1; l < nsl; ++l) {
            const SLevelDev &P = m->slv[l - 1], &L = m->slv[l];
            k_fill<T><<<grid1(sv[l].n), BS, 0, s>>>(sv[l], sv[l].n, (T)0);
            for (int tc = 0; tc < std::min(3, K); ++tc)
                for (int c = 0; c < L.ncolor; ++c) {
                    k_sprobe<T><<<grid2(P.n, K), BS, 0, s>>>(P.n, P.agg, L.color, tc, c, stt[l - 1]);
                    s_apply(st, l - 1, stt[l - 1], nullptr, sr[l - 1]);
                    k_srestrict<T><<<grid2(L.n, K), BS, 0, s>>>(L.n, P.n, P.mem_ptr, P.mem_idx, sr[l - 1], sb[l]);
                    k_sscatter<T><<<grid2(L.n, K), BS, 0, s>>>(slview(m, l), K, L.slot_of, tc, c, sb[l], sv[l]);
                }
            k_sdiag<T><<<grid2(L.n, K), BS, 0, s>>>(slview(m, l), K, sv[l], sd0, sdl, sdu);
            k_tri_factor<T><<<grid1(L.n, 1 << 20), BS, 0, s>>>(L.n, K, sd0, sdl, sdu, sinv[l], slm[l], sup[l]);
        }
    }

    // one V-cycle x = M_l^-1 b with damped time-line Jacobi smoothing
    void s_vcycle(ot_state *st, int l, const T *b, T *x) {
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        const size_t nk = (size_t)K * m->slv[l].n;
        s_tri(st, l, b, stt[l]);
        k_axpby<T><<<grid1(nk), BS, 0, s>>>(nk, somega, stt[l], 0.0, x);
        if (l == nsl - 1) {
            for (int it = 1; it < s_coarse_its; ++it) {
                s_apply(st, l, x, b, sr[l]);
                s_tri(st, l, sr[l], stt[l]);
                k_axpby<T><<<grid1(nk), BS, 0, s>>>(nk, somega, stt[l], 1.0, x);
            }
            return;
        }
        const SLevelDev &L = m->slv[l];
        for (int it = 1; it < s_nu; ++it) {
            s_apply(st, l, x, b, sr[l]);
            s_tri(st, l, sr[l], stt[l]);
            k_axpby<T><<<grid1(nk), BS, 0, s>>>(nk, somega, stt[l], 1.0, x);
        }
        s_apply(st, l, x, b, sr[l]);
        k_srestrict<T><<<grid2(L.n_next, K), BS, 0, s>>>(L.n_next, L.n, L.mem_ptr, L.mem_idx, sr[l], sb[l + 1]);
        s_vcycle(st, l + 1, sb[l + 1], sx[l + 1]);
        k_sprolong<T><<<grid2(L.n, K), BS, 0, s>>>(L.n, L.n_next, L.agg, sx[l + 1], s_alpha, x);
        for (int it = 0; it < s_nu; ++it) {
            s_apply(st, l, x, b, sr[l]);
            s_tri(st, l, sr[l], stt[l]);
            k_axpby<T><<<grid1(nk), BS, 0, s>>>(nk, somega, stt[l], 1.0, x);
        }
    }

    // preconditioner of the inner GMRES: multigrid when a hierarchy exists.
    // The system is solved row-scaled by the inverse probed diagonal, so the
    // preconditioner first undoes that scaling (x = M^-1 (d0 r)).
    void s_prec(ot_state *st, const T *r, T *x) {
        k_dscale<T><<<grid1(mrho), BS, 0, st->stream>>>(mrho, d0, 0, r, tmpm3);
        if (nsl >= 2) s_vcycle(st, 0, tmpm3, x);
        else tri_apply(st, tmpm3, x);
    }
    // scaled operator: out = D0^-1 S z
    void s_scaled_apply(ot_state *st, const T *z, T *out) {
        schur_apply(st, z, out);
        k_dscale<T><<<grid1(mrho), BS, 0, st->stream>>>(mrho, d0, 1, out, out);
    }

    LevelView lview(const ot_mesh *m, int l) const {
        const MGLevelDev &L = m->lv[l];
        LevelView v;
        v.n = L.n; v.w = L.w; v.ne = L.ne; v.nb = L.nb; v.ed = L.ed;
        return v;
    }

    // the K+1 rho~-weighted Laplacians: gradients g, multigrid edge weights
    // of every level and their inverse diagonals
    void lap_setup(ot_state *st) {
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        k_lin_edges<T><<<grid2(ne, K + 1), BS, 0, s>>>(mesh_view(m), st->view(), g, lw[0]);
        for (int l = 0; l < nlev; ++l) {
            const MGLevelDev &L = m->lv[l];
            if (l > 0) {
                const MGLevelDev &P = m->lv[l - 1];
                k_mg_coarse_w<T><<<grid2(P.ne_next, K + 1), BS, 0, s>>>(P.ne_next, P.ne, P.cedge_ptr,
                                                                         P.cedge_idx, lw[l - 1], lw[l]);
            }
            k_mg_diag<T><<<grid2(L.n, K + 1), BS, 0, s>>>(lview(m, l), lw[l], ldinv[l]);
        }
    }

    // linearisation: FP32/FP64 copies of the coefficients, multigrid
    // hierarchy weights, probed time-line tridiagonal factors
    void setup(ot_state *st) override {
        if (nf == 0) alloc(st);
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        MeshView mv = mesh_view(m);
        StateView sv = st->view();
        lap_setup(st);
        if (nce > 0) k_lin_cedges<T><<<grid2(nce, K), BS, 0, s>>>(mv, sv, wc);
        k_convert<T, double><<<grid1(mrho), BS, 0, s>>>(st->rho, rhoT, mrho);
        k_convert<T, double><<<grid1(mrho), BS, 0, s>>>(st->s, sT, mrho);
        if (tb_b < 0) autotune_schur_blocking(st);
        // probe the block-tridiagonal pseudo-Schur operator for its three
        // time diagonals at every coarse cell
        const int ncol = m->h.ncolor;
        dim3 gc = grid2(nc, K);
        k_fill<double><<<grid1(mrho), BS, 0, s>>>(dl, mrho, 0.0);
        k_fill<double><<<grid1(mrho), BS, 0, s>>>(du, mrho, 0.0);
        for (int tc = 0; tc < std::min(3, K); ++tc)
            for (int c = 0; c < ncol; ++c) {
                k_probe<T><<<gc, BS, 0, s>>>(nc, m->color, tc, c, probe);
                schur_apply(st, probe, tmpm);
                k_probe_scatter<T><<<gc, BS, 0, s>>>(nc, K, m->color, tc, c, tmpm, d0, dl, du);
            }
        k_tri_factor<T><<<grid1(nc, 1 << 20), BS, 0, s>>>(nc, K, d0, dl, du, inv_dd, lm, up);
        s_setup(st);
    }

    // out = (Diag(s) A~ - Diag(rho) B M^-1 B~) z
    void schur_apply(ot_state *st, const T *z, T *out) {
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        MeshView mv = mesh_view(m);
        k_schur_lift<T><<<grid2(nf, K + 1), BS, 0, s>>>(mv, K, z, uT);
        // time-blocked passes (levels per thread; 0 = per-level kernels) when
        // the cell stencils fit their register caps
        const int tb_btilde = blocking_fits(m) ? tb_b : 0, tb_out = blocking_fits(m) ? tb_o : 0;
        launch_btilde(st, z, tb_btilde);
        launch_out(st, z, out, tb_out);
    }

    static bool blocking_fits(const ot_mesh *m) {
        const MeshHost &h = m->h;
        return h.wf <= kTbWF && h.wo <= kTbWO && h.woc <= kTbWOC && h.wr <= kTbWR && h.wcc <= kTbWCC;
    }

    // pass 2 of the pseudo-Schur operator, v = M^-1 B~ z (u from pass 1)
    void launch_btilde(ot_state *st, const T *z, int tb_btilde) {
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        MeshView mv = mesh_view(m);
        const double b = sizeof(T), S1 = K + 1;
        const MeshHost &h = m->h;
        {
            // z, u, g, v once; overlap, cell-edge and edge geometry once
            const double bytes = b * ((double)K * nc + 2.0 * S1 * nf + S1 * ne) +
                                 12.0 * h.wo * nf + 8.0 * h.wf * nf + 28.0 * ne + 8.0 * nf;
            const kprof::Ev ev = kprof::take(OT_KPROF_SCHUR_BTILDE, sizeof(T), bytes);
            if (tb_btilde > 0)
                hipExtLaunchKernelGGL(k_schur_btilde_tb<T>, dim3(ceil_div(nf, BS), ceil_div(K + 1, tb_btilde)),
                                      dim3(BS), 0, s, ev.a, ev.b, 0, mv, K, tb_btilde, st->dt, z, (const T *)uT.p,
                                      (const T *)g.p, vT.p);
            else
                hipExtLaunchKernelGGL(k_schur_btilde<T>, grid2(nf, K + 1), dim3(BS), 0, s, ev.a, ev.b, 0, mv, K,
                                      st->dt, z, (const T *)uT.p, (const T *)g.p, vT.p);
        }
    }

    // pass 3, out = s (A~ z) - rho (B v)
    void launch_out(ot_state *st, const T *z, T *out, int tb_out) {
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        MeshView mv = mesh_view(m);
        const double b = sizeof(T), S1 = K + 1;
        const MeshHost &h = m->h;
        {
            // z, v, g, w~, rho, s, out once; coarse-cell geometry once
            const double bytes = b * (4.0 * K * nc + S1 * nf + S1 * ne + (double)K * nce) + 8.0 * h.wcc * nc +
                                 12.0 * h.woc * nc + 20.0 * h.wr * nc;
            const kprof::Ev ev = kprof::take(OT_KPROF_SCHUR_OUT, sizeof(T), bytes);
            if (tb_out > 0)
                hipExtLaunchKernelGGL(k_schur_out_tb<T>, dim3(ceil_div(nc, BS), ceil_div(K, tb_out)), dim3(BS),
                                      0, s, ev.a, ev.b, 0, mv, K, tb_out, st->dt, z, (const T *)vT.p,
                                      (const T *)g.p, (const T *)wc.p, (const T *)rhoT.p, (const T *)sT.p, out);
            else
                hipExtLaunchKernelGGL(k_schur_out<T>, grid2(nc, K), dim3(BS), 0, s, ev.a, ev.b, 0, mv, K, st->dt,
                                      z, (const T *)vT.p, (const T *)g.p, (const T *)wc.p, (const T *)rhoT.p,
                                      (const T *)sT.p, out);
        }
    }

    // Autotuner of the time blocking (levels per thread) of passes 2 and 3:
    // each candidate is timed with HIP events on this preconditioner's own
    // mesh, K and precision (3 launches each, after one untimed launch) and
    // the fastest kept.  Runs once, at the first linearisation.
    void autotune_schur_blocking(ot_state *st) {
        const int r = sizeof(T) == 8 ? 1 : 0;
        tb_b = g_schur_tb[r][0];
        tb_o = g_schur_tb[r][1];
        if (g_schur_tb_fixed[r] || !blocking_fits(st->mesh)) return;
        const auto key = std::make_tuple(nf, nc, ne, K, r);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                tb_b = it->second.first;
                tb_o = it->second.second;
                return;
            }
        }
        hipStream_t s = st->stream;
        k_fill<T><<<grid1(mrho), BS, 0, s>>>(probe, mrho, (T)1);
        k_schur_lift<T><<<grid2(nf, K + 1), BS, 0, s>>>(mesh_view(st->mesh), K, probe, uT);
        hipEvent_t e0, e1;
        OT_HIP(hipEventCreate(&e0));
        OT_HIP(hipEventCreate(&e1));
        auto time_it = [&](const std::function<void()> &f) {
            f();
            OT_HIP(hipEventRecord(e0, s));
            for (int rep = 0; rep < 3; ++rep) f();
            OT_HIP(hipEventRecord(e1, s));
            OT_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            OT_HIP(hipEventElapsedTime(&ms, e0, e1));
            return ms;
        };
        const int cand[] = {0, 4, 8, 16, 32};
        float best_b = 1e30f, best_o = 1e30f;
        for (int c : cand) {
            if (c > K + 1) continue;
            const float tb = time_it([&] { launch_btilde(st, probe, c); });
            if (tb < best_b) { best_b = tb; tb_b = c; }
        }
        for (int c : cand) {
            if (c > K) continue;
            const float to = time_it([&] { launch_out(st, probe, tmpm, c); });
            if (to < best_o) { best_o = to; tb_o = c; }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        {
            // a state of the same shape tuned meanwhile: adopt its choice
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto ins = g_tune_cache.emplace(key, std::make_pair(tb_b, tb_o));
            tb_b = ins.first->second.first;
            tb_o = ins.first->second.second;
        }
        if (st->opt.verbose)
            fprintf(stderr, "  pseudo-Schur blocking (%s): M^-1 B~ pass %d levels/thread (%.1f us), output pass %d "
                    "(%.1f us)\n", sizeof(T) == 8 ? "FP64" : "FP32", tb_b, 1000.0f * best_b / 3, tb_o,
                    1000.0f * best_o / 3);
    }

    // time-line tridiagonal solve of n cells: one wavefront per cell with a
    // scan over time (K <= kTriScanMaxK), else one thread per cell
    template <int FINE>
    void tri_launch(hipStream_t s, int n, const T *dinv, const T *l, const T *u, const T *r, T *x, kprof::Ev ev) {
        if (K <= kTriScanMaxK)
            hipExtLaunchKernelGGL(k_tri_scan<T, FINE>, dim3(ceil_div(n, BS / 64)), dim3(BS), 0, s, ev.a, ev.b, 0,
                                  n, K, dinv, l, u, r, x);
        else
            hipExtLaunchKernelGGL(k_tri_solve<T, FINE>, dim3(grid1(n, 1 << 20)), dim3(BS), 0, s, ev.a, ev.b, 0,
                                  n, K, dinv, l, u, r, x);
    }

    void tri_apply(ot_state *st, const T *r, T *x) {
        // reads r, l, u, 1/d; writes x (all K x nc)
        const kprof::Ev ev = kprof::take(OT_KPROF_TRI_FINE, sizeof(T), 5.0 * sizeof(T) * (double)K * nc);
        tri_launch<1>(st->stream, nc, inv_dd, lm, up, r, x, ev);
    }

    // right-preconditioned restarted GMRES on the pseudo-Schur system; w = 0
    // start.  The Krylov basis, the scaled right-hand side and the
    // Gram-Schmidt updates are FP64 in both paths; with T = float only the
    // operator and the V-cycle run in FP32 (their inputs and outputs are
    // converted).  An FP32 basis loses orthogonality within a few tens of
    // iterations when the new direction nearly lies in the span (its norm
    // after orthogonalisation far below its norm before): on the 256^2,
    // K = 64 benchmark the outer FGMRES then needed 4-5x the FP64 path's
    // iterations on the early Newton systems, and more inner iterations
    // made it worse.
    int gmres_schur(ot_state *st, const T *rhs, T *w, double tol, int maxit) {
        hipStream_t s = st->stream;
        const size_t n = mrho;
        constexpr bool f64 = std::is_same<T, double>::value;
        k_fill<T><<<grid1(n), BS, 0, s>>>(w, n, (T)0);
        // row scaling by the inverse diagonal: the rows of near-empty cells
        // (s A~ dominated) and of dense cells (rho-weighted time Laplacian)
        // differ by orders of magnitude
        if constexpr (f64) {
            k_dscale<double><<<grid1(n), BS, 0, s>>>(n, d0, 1, rhs, rhsc);
        } else {
            k_convert<double, T><<<grid1(n), BS, 0, s>>>(rhs, rhsc.p, n);
            k_dscale<double><<<grid1(n), BS, 0, s>>>(n, d0, 1, rhsc, rhsc);
        }
        const double *rs = rhsc.p;
        double beta = norm2<double>(st, rs, n);
        if (beta == 0.0) return 0;
        const double target = tol * beta;
        Givens G(mS);
        int its = 0;
        // operator input in T: the FP64 vector itself, or its FP32 copy
        auto in_T = [&](const double *x) -> const T * {
            if constexpr (f64) return x;
            else {
                k_convert<T, double><<<grid1(n), BS, 0, s>>>(x, tmpm2.p, n);
                return tmpm2.p;
            }
        };
        // D0^-1 S z into the FP64 vector out
        auto scaled_apply_to = [&](const T *z, double *out) {
            if constexpr (f64) s_scaled_apply(st, z, out);
            else {
                s_scaled_apply(st, z, tmpm2.p);
                k_convert<double, T><<<grid1(n), BS, 0, s>>>(tmpm2.p, out, n);
            }
        };
        // r = rhs (w = 0)
        k_convert<double, double><<<grid1(n), BS, 0, s>>>(rs, VS.p, n);
        double res = beta;
        while (its < maxit) {
            k_axpby<double><<<grid1(n), BS, 0, s>>>(n, 0.0, VS.p, 1.0 / beta, VS.p);
            G.reset(beta);
            int j = 0;
            std::vector<double> h(mS + 1);
            for (; j < mS && its < maxit; ++j) {
                s_prec(st, in_T(VS.p + (size_t)j * n), tmpm);
                double *wn = VS.p + (size_t)(j + 1) * n;
                scaled_apply_to(tmpm, wn);
                double hn = cgs2<double>(st, VS.p, n, j + 1, wn, n, h.data());
                for (int i = 0; i <= j; ++i) G.h(i, j) = h[i];
                G.h(j + 1, j) = hn;
                ++its;
                res = G.push(j);
                if (hn > 0) k_axpby<double><<<grid1(n), BS, 0, s>>>(n, 0.0, wn, 1.0 / hn, wn);
                if (res <= target || hn == 0.0) { ++j; break; }
            }
            std::vector<double> y = G.solve(j);
            DBuf<double> &yd = st->shift;      // small device scratch (>= mS)
            OT_HIP(hipMemcpyAsync(yd.p, y.data(), j * sizeof(double), hipMemcpyHostToDevice, s));
            k_combine<double, T><<<grid1(n), BS, 0, s>>>(n, VS.p, n, j, yd.p, 0.0, tmpm2.p);
            s_prec(st, tmpm2, tmpm);
            k_axpby<T><<<grid1(n), BS, 0, s>>>(n, 1.0, tmpm, 1.0, w);
            OT_HIP(hipStreamSynchronize(s));   // y lives in pageable host memory
            if (res <= target || its >= maxit) break;
            // restart: r = D0^-1 (rhs - S w)
            scaled_apply_to(w, VS.p);
            k_axpby<double><<<grid1(n), BS, 0, s>>>(n, 1.0, rs, -1.0, VS.p);
            beta = norm2<double>(st, VS.p, n);
            if (beta <= target) break;
        }
        return its;
    }

    // ---- multigrid V-cycle on all K+1 slices at level l: x = M_l^-1 b
    void cheb(ot_state *st, int l, const T *b, T *x, bool zero_x, int deg, double lo) {
        const ot_mesh *m = st->mesh;
        LevelView L = lview(m, l);
        hipStream_t s = st->stream;
        dim3 gr = grid2(L.n, K + 1);
        const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
        k_cheb_init<T><<<gr, BS, 0, s>>>(L, lw[l], ldinv[l], b, x, lr[l], ld[l], theta, zero_x ? 1 : 0);
        double rho_old = 1.0 / sigma;
        T *d = ld[l], *d2 = ld2[l];
        for (int it = 0; it < deg; ++it) {
            const double rho_new = 1.0 / (2.0 * sigma - rho_old);
            if (l == 0) {
                // x, r read and written; d, 1/D read; d' written; weights and ELL once
                const double S1 = K + 1;
                const kprof::Ev ev =
                    kprof::take(OT_KPROF_CHEB_FINE, sizeof(T), sizeof(T) * (7.0 * S1 * L.n + S1 * L.ne) + 8.0 * L.w * L.n);
                hipExtLaunchKernelGGL(k_cheb_step<T, 1>, gr, dim3(BS), 0, s, ev.a, ev.b, 0, L, (const T *)lw[l].p,
                                      (const T *)ldinv[l].p, x, lr[l].p, (const T *)d, d2, rho_new * rho_old,
                                      2.0 * rho_new / delta);
            } else {
                k_cheb_step<T><<<gr, BS, 0, s>>>(L, lw[l], ldinv[l], x, lr[l], d, d2, rho_new * rho_old,
                                                 2.0 * rho_new / delta);
            }
            rho_old = rho_new;
            std::swap(d, d2);
        }
    }

    void vcycle(ot_state *st, int l, const T *b, T *x) {
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        if (l == nlev - 1) {
            cheb(st, l, b, x, true, coarse_deg, coarse_lo_ratio * hi);
            return;
        }
        const MGLevelDev &Lv = m->lv[l];
        cheb(st, l, b, x, true, nu, lo_ratio * hi);
        k_mg_restrict<T><<<grid2(Lv.n_next, K + 1), BS, 0, s>>>(lview(m, l), Lv.n_next, Lv.mem_ptr, Lv.mem_idx,
                                                                lw[l], b, x, lb[l + 1]);
        vcycle(st, l + 1, lb[l + 1], lx[l + 1]);
        k_mg_prolong<T><<<grid2(Lv.n, K + 1), BS, 0, s>>>(Lv.n, Lv.n_next, Lv.agg, lx[l + 1], x, mg_alpha);
        cheb(st, l, b, x, false, nu, lo_ratio * hi);
    }

    // PCG on the K+1 slices A^k x^k = b^k (b already zero-mean); x zero-mean on exit
    // preconditioner of the PCG: one T-precision V-cycle z = M^-1 r
    void pcg_prec(ot_state *st, const double *r, double *z) {
        hipStream_t s = st->stream;
        k_convert<T, double><<<grid1(nphi), BS, 0, s>>>(r, vb, nphi);
        vcycle(st, 0, vb, vx);
        k_convert<double, T><<<grid1(nphi), BS, 0, s>>>(vx, z, nphi);
    }

    int pcg(ot_state *st, const T *b, double *x, double tol, int maxit) {
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        const int S = K + 1;
        LevelView L0 = lview(m, 0);
        dim3 gr = grid2(nf, S);
        double *dsum = st->sums.p;               // scratch (>= S)
        k_fill<double><<<grid1(nphi), BS, 0, s>>>(x, nphi, 0.0);
        k_convert<double, T><<<grid1(nphi), BS, 0, s>>>(b, pr.p, nphi);
        std::vector<double> bn(S), rz(S), alpha(S), beta(S);
        std::vector<char> active(S, 1);
        {
            const double *h = st->red.fetch(slice_dots<double>(st, pr.p, pr.p, nf, S, dsum), S);
            for (int k = 0; k < S; ++k) { bn[k] = std::sqrt(h[k]); active[k] = bn[k] > 0.0; }
        }
        if (std::none_of(active.begin(), active.end(), [](char c) { return c; })) return 0;
        pcg_prec(st, pr, pz);
        {
            const double *h = st->red.fetch(slice_dots<double>(st, pr.p, pz.p, nf, S, dsum), S);
            for (int k = 0; k < S; ++k) rz[k] = h[k];
        }
        k_convert<double, double><<<grid1(nphi), BS, 0, s>>>(pz.p, pp.p, nphi);
        int it = 0;
        for (it = 1; it <= maxit; ++it) {
            k_mg_apply<T, double><<<gr, BS, 0, s>>>(L0, lw[0], pp, pq);
            const double *h = st->red.fetch(slice_dots<double>(st, pp.p, pq.p, nf, S, dsum), S);
            for (int k = 0; k < S; ++k) alpha[k] = (active[k] && h[k] > 0.0) ? rz[k] / h[k] : 0.0;
            OT_HIP(hipMemcpyAsync(coef.p, alpha.data(), S * sizeof(double), hipMemcpyHostToDevice, s));
            k_pcg_xr<double><<<gr, BS, 0, s>>>(nf, coef, pp, pq, x, pr);
            const double *h2 = st->red.fetch(slice_dots<double>(st, pr.p, pr.p, nf, S, dsum), S);
            bool any = false;
            for (int k = 0; k < S; ++k) {
                if (active[k] && std::sqrt(std::max(h2[k], 0.0)) <= tol * bn[k]) active[k] = 0;
                any = any || active[k];
            }
            if (!any) break;
            pcg_prec(st, pr, pz);
            const double *h3 = st->red.fetch(slice_dots<double>(st, pr.p, pz.p, nf, S, dsum), S);
            for (int k = 0; k < S; ++k) {
                beta[k] = (active[k] && rz[k] != 0.0) ? h3[k] / rz[k] : 0.0;
                if (active[k]) rz[k] = h3[k];
            }
            OT_HIP(hipMemcpyAsync(coef.p + S, beta.data(), S * sizeof(double), hipMemcpyHostToDevice, s));
            k_pcg_p<double><<<gr, BS, 0, s>>>(nf, coef.p + S, pz, pp);
        }
        OT_HIP(hipStreamSynchronize(s));
        return std::min(it, maxit);
    }

    void schur_apply_d(ot_state *st, const double *z, double *out) override {
        k_convert<T, double><<<grid1(mrho), BS, 0, st->stream>>>(z, tmpm2, mrho);
        schur_apply(st, tmpm2, probe);
        k_convert<double, T><<<grid1(mrho), BS, 0, st->stream>>>(probe, out, mrho);
    }
    int schur_solve_d(ot_state *st, const double *rhs, double *z, double tol, int maxit) override {
        k_convert<T, double><<<grid1(mrho), BS, 0, st->stream>>>(rhs, rhsS, mrho);
        int its = gmres_schur(st, rhsS, zS, tol, maxit);
        k_convert<double, T><<<grid1(mrho), BS, 0, st->stream>>>(zS, z, mrho);
        return its;
    }
    void tri_solve_d(ot_state *st, const double *r, double *x) override {
        k_convert<T, double><<<grid1(mrho), BS, 0, st->stream>>>(r, tmpm3, mrho);
        tri_apply(st, tmpm3, tmpm2);
        k_convert<double, T><<<grid1(mrho), BS, 0, st->stream>>>(tmpm2, x, mrho);
    }
    void tri_diagonals_d(ot_state *st, double *a0, double *al, double *au) override {
        OT_HIP(hipMemcpyAsync(a0, d0.p, mrho * sizeof(double), hipMemcpyDeviceToDevice, st->stream));
        OT_HIP(hipMemcpyAsync(al, dl.p, mrho * sizeof(double), hipMemcpyDeviceToDevice, st->stream));
        OT_HIP(hipMemcpyAsync(au, du.p, mrho * sizeof(double), hipMemcpyDeviceToDevice, st->stream));
    }
    int laplace_solve_d(ot_state *st, const double *b, double *x, double tol, int maxit) override {
        k_convert<T, double><<<grid1(nphi), BS, 0, st->stream>>>(b, bT, nphi);
        int its = pcg(st, bT, px, tol, maxit);
        k_convert<double, double><<<grid1(nphi), BS, 0, st->stream>>>(px, x, nphi);
        return its;
    }
    size_t level_data_d(ot_state *st, int level, int what, double *out) override {
        OT_REQUIRE(level >= 0 && level < nlev, OT_EINVAL, "bad level");
        const MGLevelDev &L = st->mesh->lv[level];
        const size_t n = (size_t)(K + 1) * (what == 0 ? L.ne : L.n);
        if (out) k_convert<double, T><<<grid1(n), BS, 0, st->stream>>>(what == 0 ? lw[level] : ldinv[level], out, n);
        return n;
    }
    void vcycle_d(ot_state *st, const double *b, double *x) override {
        k_convert<T, double><<<grid1(nphi), BS, 0, st->stream>>>(b, vb, nphi);
        vcycle(st, 0, vb, vx);
        k_convert<double, T><<<grid1(nphi), BS, 0, st->stream>>>(vx, x, nphi);
    }

    // z = P_BB^-1 r (FP64 in/out)
    void apply(ot_state *st, const double *r, double *z) override {
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        const double tolS = st->opt.eps_in_S, tolA = st->opt.eps_in_A;
        const int maxit = st->opt.max_inner;
        k_convert<T, double><<<grid1(nphi), BS, 0, s>>>(r, cT, nphi);
        k_convert<T, double><<<grid1(mrho), BS, 0, s>>>(r + nphi, dT, mrho);
        // (i) pseudo-Schur solve
        double *dsum = st->sums.p + 2 * (K + 2);
        slice_sums<T>(st, dT.p, nullptr, nc, K, dsum);
        dim3 gc = grid2(nc, K);
        k_schur_rhs<T><<<gc, BS, 0, s>>>(m->ac, nc, st->area, dsum, rhoT, dT, rhsS);
        st->acc.inner_S_iters += gmres_schur(st, rhsS, zS, tolS, st->opt.max_inner_S);
        // (ii) y = P^T M'^-1 A~ z
        k_coarse_lap_scaled<T><<<gc, BS, 0, s>>>(mesh_view(m), zS, wc, yT);
        double *ys = st->sums.p + 3 * (K + 2);
        slice_sums<T>(st, yT.p, m->ac, nc, K, ys);
        k_slice_shift<T><<<gc, BS, 0, s>>>(nc, ys, 1.0 / st->area, yT);
        // (iii) b = c - B^T y, projected to zero sum per slice
        dim3 gf = grid2(nf, K + 1);
        k_bt_rhs<T><<<gf, BS, 0, s>>>(mesh_view(m), K, st->dt, cT, yT, g, bT);
        double *bs = st->sums.p + 4 * (K + 2);
        slice_sums<T>(st, bT.p, nullptr, nf, K + 1, bs);
        k_slice_shift<T><<<gf, BS, 0, s>>>(nf, bs, 1.0 / nf, bT);
        // (iv) K+1 Laplacian solves, zero-sum solutions
        st->acc.inner_A_iters += pcg(st, bT, px, tolA, maxit);
        slice_sums<double>(st, px.p, nullptr, nf, K + 1, bs);
        k_slice_shift<double><<<gf, BS, 0, s>>>(nf, bs, 1.0 / nf, px);
        k_convert<double, double><<<grid1(nphi), BS, 0, s>>>(px, z, nphi);
        k_convert<double, T><<<grid1(mrho), BS, 0, s>>>(yT, z + nphi, mrho);
        st->acc.prec_applies++;
    }
};

// ---------------------------------------------------------------------------
// SIMPLE preconditioner (Sec. 4.3) on the projected system, FP64
// ---------------------------------------------------------------------------
// P^-1 (c; d): u = D^-1 c with D = Diag(A); v = d - P B u; y solves
// P (C + B D^-1 B^T) P^T y = -v (the negative of the approximate Schur
// complement S~ = -(C + B D^-1 B^T), projected); x = u - D^-1 B^T P^T y.
// The inner system is symmetric positive semidefinite with the per-slice
// constants as kernel and a consistent right-hand side; it is solved by PCG
// to eps_in_S (cap max_inner) preconditioned by the exact time-line
// tridiagonal part T of C + B D^-1 B^T (probed, like the pseudo-Schur time
// diagonals of the BB preconditioner), applied in the form consistent with
// the projection (ctri).
struct SimplePrec : PrecBase {
    int nf = 0, nc = 0, K = 0;
    size_t nphi = 0, mrho = 0;
    DBuf<double> dA, u, tphi, bu, v, y, r, z, p, q, w, probe, d0, dl, du, inv_dd, lm, up, zsum;
    DBuf<double> gmat, ginv, lam;              // K x K slice coupling of the constrained time-line solve

    void alloc(ot_state *st) {
        const ot_mesh *m = st->mesh;
        nf = m->h.nf; nc = m->h.nc; K = st->K;
        nphi = st->nphi; mrho = st->mrho;
        dA.alloc(nphi); u.alloc(nphi); tphi.alloc(nphi);
        for (DBuf<double> *b : {&bu, &v, &y, &r, &z, &p, &q, &w, &probe, &d0, &dl, &du, &inv_dd, &lm, &up})
            b->alloc(mrho);
        zsum.alloc(K + 2);
        gmat.alloc((size_t)K * K);
        lam.alloc(K + 2);
    }

    // out = (C + B D^-1 B^T) P^T x (project = true) or (C + B D^-1 B^T) x,
    // then P applied to the result when project is set
    void opX(ot_state *st, const double *x, double *out, bool project) {
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        MeshView mv = mesh_view(m);
        StateView sv = st->view();
        double *cs = st->sums.p + 5 * (K + 2);           // a'^T x^k (for P^T x)
        if (project) slice_sums<double>(st, x, m->ac, nc, K, cs);
        else k_fill<double><<<1, BS, 0, s>>>(cs, K + 2, 0.0);
        k_saddle_phi<<<grid2(nf, K + 1), BS, 0, s>>>(mv, sv, nullptr, x, cs, dA, tphi.p);  // D^-1 B^T P^T x
        dim3 gc = grid2(nc, K);
        k_opB<<<gc, BS, 0, s>>>(mv, sv, tphi, x, cs, -1.0, out, st->red.part);              // B (.) + C P^T x
        if (project) {
            double *us = st->sums.p + 6 * (K + 2);
            k_seg_final<<<K, BS, 0, s>>>(st->red.part, gc.x, us);
            k_proj_fix<double><<<gc, BS, 0, s>>>(m->ac, nc, us, st->area, out);
        }
    }

    void setup(ot_state *st) override {
        if (nf == 0) alloc(st);
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        k_lap_diag<<<grid2(nf, K + 1), BS, 0, s>>>(mesh_view(m), st->view(), dA);
        // time-line tridiagonal part of C + B D^-1 B^T by probing (the colouring
        // separates cells coupled through the fine cells around their overlaps)
        dim3 gc = grid2(nc, K);
        k_fill<double><<<grid1(mrho), BS, 0, s>>>(dl, mrho, 0.0);
        k_fill<double><<<grid1(mrho), BS, 0, s>>>(du, mrho, 0.0);
        for (int tc = 0; tc < std::min(3, K); ++tc)
            for (int c = 0; c < m->h.ncolor; ++c) {
                k_probe<double><<<gc, BS, 0, s>>>(nc, m->color, tc, c, probe);
                opX(st, probe, q, false);
                k_probe_scatter<double><<<gc, BS, 0, s>>>(nc, K, m->color, tc, c, q, d0, dl, du);
            }
        k_tri_factor<double><<<grid1(nc, 1 << 20), BS, 0, s>>>(nc, K, d0, dl, du, inv_dd, lm, up);
        // G[l][k] = a'^T (T^-1 a'_l)^k, a'_l the coarse areas on slice l: the
        // slice coupling of the constrained time-line solve (ctri)
        for (int l = 0; l < K; ++l) {
            k_fill<double><<<grid1(mrho), BS, 0, s>>>(probe, mrho, 0.0);
            OT_HIP(hipMemcpyAsync(probe.p + (size_t)l * nc, m->ac, nc * sizeof(double), hipMemcpyDeviceToDevice, s));
            tri(st, probe, q);
            slice_sums<double>(st, q.p, m->ac, nc, K, gmat.p + (size_t)l * K);
        }
        std::vector<double> G((size_t)K * K);
        OT_HIP(hipMemcpyAsync(G.data(), gmat.p, G.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        OT_HIP(hipStreamSynchronize(s));
        ginv.upload(spd_inverse(G, K), s);
        OT_HIP(hipStreamSynchronize(s));
    }

    // Inverse of a small symmetric positive definite matrix (row-major) by
    // Cholesky; G above is SPD because T is (a principal part of the SPD
    // C + B D^-1 B^T) and the a'_l are independent.
    static std::vector<double> spd_inverse(const std::vector<double> &A, int n) {
        std::vector<double> L((size_t)n * n, 0.0), X((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j <= i; ++j) {
                double v = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
                for (int q = 0; q < j; ++q) v -= L[(size_t)i * n + q] * L[(size_t)j * n + q];
                if (i == j) {
                    OT_REQUIRE(v > 0.0, OT_ELINSOLVE, "SIMPLE: slice coupling of the time-line solve not positive");
                    L[(size_t)i * n + i] = std::sqrt(v);
                } else {
                    L[(size_t)i * n + j] = v / L[(size_t)j * n + j];
                }
            }
        for (int c = 0; c < n; ++c) {               // solve L L^T x = e_c
            std::vector<double> y(n, 0.0);
            for (int i = 0; i < n; ++i) {
                double v = i == c ? 1.0 : 0.0;
                for (int q = 0; q < i; ++q) v -= L[(size_t)i * n + q] * y[q];
                y[i] = v / L[(size_t)i * n + i];
            }
            for (int i = n - 1; i >= 0; --i) {
                double v = y[i];
                for (int q = i + 1; q < n; ++q) v -= L[(size_t)q * n + i] * X[(size_t)q * n + c];
                X[(size_t)i * n + c] = v / L[(size_t)i * n + i];
            }
        }
        return X;
    }

    // Time-line preconditioner made consistent with the projection: for r in
    // range(P), x = T^-1 (r - a' lam) with lam = G^-1 (a'^T T^-1 r), so that
    // a'^T x^k = 0 on every slice (x in range(P^T), where P X P^T acts as
    // P X).  The plain T^-1 ignores the projection and leaves PCG several
    // times slower on P X P^T.
    void ctri(ot_state *st, const double *rr, double *x) {
        hipStream_t s = st->stream;
        const ot_mesh *m = st->mesh;
        tri(st, rr, x);
        slice_sums<double>(st, x, m->ac, nc, K, zsum.p);
        k_small_gemv<<<1, BS, 0, s>>>(K, ginv, zsum, lam);
        k_sub_slice_cols<<<grid2(nc, K), BS, 0, s>>>(nc, m->ac, lam, rr, w);
        tri(st, w, x);
    }

    void tri(ot_state *st, const double *rr, double *x) {
        if (K <= kTriScanMaxK)
            k_tri_scan<double, 0><<<ceil_div(nc, BS / 64), BS, 0, st->stream>>>(nc, K, inv_dd, lm, up, rr, x);
        else
            k_tri_solve<double, 0><<<grid1(nc, 1 << 20), BS, 0, st->stream>>>(nc, K, inv_dd, lm, up, rr, x);
    }

    double dot(ot_state *st, const double *a, const double *b) {
        double *out = st->sums.p + 7 * (K + 2);
        const int nblk = std::min(256, std::max(1, ceil_div((int64_t)mrho, BS)));
        k_seg_dot_partial<double><<<dim3(nblk, 1), BS, 0, st->stream>>>(a, b, (int)mrho, st->red.part);
        k_seg_final<<<1, BS, 0, st->stream>>>(st->red.part, nblk, out);
        return st->red.fetch(out, 1)[0];
    }

    // (a . b, a . c) with one host wait
    void dot2(ot_state *st, const double *a, const double *b, const double *c, double *ab, double *ac) {
        double *out = st->sums.p + 7 * (K + 2);
        const int nblk = std::min(256, std::max(1, ceil_div((int64_t)mrho, BS)));
        k_seg_dot_partial<double><<<dim3(nblk, 1), BS, 0, st->stream>>>(a, b, (int)mrho, st->red.part);
        k_seg_dot_partial<double><<<dim3(nblk, 1), BS, 0, st->stream>>>(a, c, (int)mrho, st->red.part.p + nblk);
        k_seg_final<<<2, BS, 0, st->stream>>>(st->red.part, nblk, out);
        const double *h = st->red.fetch(out, 2);
        *ab = h[0];
        *ac = h[1];
    }

    // PCG on P X P^T y = b (b consistent), y = 0 start; returns iterations
    int pcg(ot_state *st, const double *b, double tol, int maxit) {
        hipStream_t s = st->stream;
        k_fill<double><<<grid1(mrho), BS, 0, s>>>(y, mrho, 0.0);
        k_convert<double, double><<<grid1(mrho), BS, 0, s>>>(b, r, mrho);
        const double bn = std::sqrt(std::max(dot(st, r, r), 0.0));
        if (bn == 0.0) return 0;
        ctri(st, r, z);
        k_convert<double, double><<<grid1(mrho), BS, 0, s>>>(z, p, mrho);
        double rz = dot(st, r, z);
        int it = 0;
        for (it = 1; it <= maxit; ++it) {
            opX(st, p, q, true);
            const double pq = dot(st, p, q);
            if (!(pq > 0.0)) break;
            const double alpha = rz / pq;
            k_cg_update<<<grid1(mrho), BS, 0, s>>>(mrho, alpha, p, q, y, r);
            ctri(st, r, z);
            double rr2, rz2;
            dot2(st, r, r, z, &rr2, &rz2);                 // one host wait for both
            if (std::sqrt(std::max(rr2, 0.0)) <= tol * bn) break;
            k_axpby<double><<<grid1(mrho), BS, 0, s>>>(mrho, 1.0, z, rz2 / rz, p);
            rz = rz2;
        }
        return std::min(it, maxit);
    }

    void apply(ot_state *st, const double *rin, double *zout) override {
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        MeshView mv = mesh_view(m);
        StateView sv = st->view();
        dim3 gc = grid2(nc, K);
        // u = D^-1 c; v = -(d - P B u) (the right-hand side of P X P^T y = -v)
        k_dscale<double><<<grid1(nphi), BS, 0, s>>>(nphi, dA, 1, rin, u);
        k_opB<<<gc, BS, 0, s>>>(mv, sv, u, nullptr, nullptr, 0.0, bu, st->red.part);
        double *us = st->sums.p + 4 * (K + 2);
        k_seg_final<<<K, BS, 0, s>>>(st->red.part, gc.x, us);
        k_proj_fix<double><<<gc, BS, 0, s>>>(m->ac, nc, us, st->area, bu.p);              // P B u
        k_convert<double, double><<<grid1(mrho), BS, 0, s>>>(bu, v, mrho);
        k_axpby<double><<<grid1(mrho), BS, 0, s>>>(mrho, -1.0, rin + nphi, 1.0, v);       // P B u - d
        st->acc.inner_S_iters += pcg(st, v, st->opt.eps_in_S, st->opt.max_inner);
        // x = u - D^-1 B^T P^T y; z = (x; y)
        double *cs = st->sums.p + 5 * (K + 2);
        slice_sums<double>(st, y.p, m->ac, nc, K, cs);
        k_saddle_phi<<<grid2(nf, K + 1), BS, 0, s>>>(mv, sv, nullptr, y, cs, dA, tphi.p);
        k_convert<double, double><<<grid1(nphi), BS, 0, s>>>(u, zout, nphi);
        k_axpby<double><<<grid1(nphi), BS, 0, s>>>(nphi, -1.0, tphi, 1.0, zout);
        k_convert<double, double><<<grid1(mrho), BS, 0, s>>>(y, zout + nphi, mrho);
        st->acc.prec_applies++;
    }

    // component access of the BB preconditioner: not part of SIMPLE
    void schur_apply_d(ot_state *, const double *, double *) override { unsupported(); }
    int schur_solve_d(ot_state *, const double *, double *, double, int) override { unsupported(); return 0; }
    void tri_diagonals_d(ot_state *, double *, double *, double *) override { unsupported(); }
    void tri_solve_d(ot_state *, const double *, double *) override { unsupported(); }
    int laplace_solve_d(ot_state *, const double *, double *, double, int) override { unsupported(); return 0; }
    void vcycle_d(ot_state *, const double *, double *) override { unsupported(); }
    size_t level_data_d(ot_state *, int, int, double *) override { unsupported(); return 0; }
    static void unsupported() {
        throw OtError(OT_EINVAL, "inspection call of the BB preconditioner on a state using SIMPLE");
    }
};

// ---------------------------------------------------------------------------
// Primal-Schur preconditioner (Sec. 4.2) on the projected system, FP64
// ---------------------------------------------------------------------------
// The block factorisation on S_p = A + B^T P^T C^-1 P B with the diagonal
// C kept in the (2,2) block: the exact inverse of [[A, B^T P^T], [P B, -C]],
// which differs from J_P only in C - P C P^T.  P^-1 (f; g):
// t = f + B^T P^T C^-1 g made zero-sum per slice; x solves S_p x = t by PCG
// to eps_in_S (cap max_inner), zero-sum per slice (S_p has the per-slice
// constants as kernel); y = C^-1 (P B x - g).  The paper solves S_p with
// AGMG; here one V-cycle of the K+1 rho~-weighted Laplacian multigrid of
// the BB preconditioner (which sees A, not B^T P^T C^-1 P B) preconditions
// the PCG.  A negative control: S_p is an anisotropic space-time operator
// whose time coupling the Laplacian multigrid does not see.
struct PrimalPrec : BBPrec<double> {
    DBuf<double> cdg, t, xs, pr2, pz2, pp2, pq2, ub, vr;

    void alloc_primal() {
        cdg.alloc(mrho); ub.alloc(mrho); vr.alloc(mrho);
        for (DBuf<double> *b : {&t, &xs, &pr2, &pz2, &pp2, &pq2}) b->alloc(nphi);
    }

    void setup(ot_state *st) override {
        if (nf == 0) {
            alloc(st);
            alloc_primal();
        }
        lap_setup(st);
        k_c_diag<<<grid2(nc, K), BS, 0, st->stream>>>(nc, st->mesh->ac, st->view(), cdg);
    }

    // out = P B x (out has m_rho entries)
    void pb(ot_state *st, const double *x, double *out) {
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        dim3 gc = grid2(nc, K);
        k_opB<<<gc, BS, 0, s>>>(mesh_view(m), st->view(), x, nullptr, nullptr, 0.0, out, st->red.part);
        double *us = st->sums.p + 4 * (K + 2);
        k_seg_final<<<K, BS, 0, s>>>(st->red.part, gc.x, us);
        k_proj_fix<double><<<gc, BS, 0, s>>>(m->ac, nc, us, st->area, out);
    }

    // out = xphi-part A x + B^T P^T v (x may be null: B^T P^T v only)
    void saddle_phi(ot_state *st, const double *x, const double *v, double *out) {
        const ot_mesh *m = st->mesh;
        double *cs = st->sums.p + 5 * (K + 2);
        slice_sums<double>(st, v, m->ac, nc, K, cs);
        k_saddle_phi<<<grid2(nf, K + 1), BS, 0, st->stream>>>(mesh_view(m), st->view(), x, v, cs, nullptr, out);
    }

    // out = S_p x = A x + B^T P^T C^-1 P B x
    void sp_apply(ot_state *st, const double *x, double *out) {
        pb(st, x, ub);
        k_dscale<double><<<grid1(mrho), BS, 0, st->stream>>>(mrho, cdg, 1, ub, vr);
        saddle_phi(st, x, vr, out);
    }

    void zero_sum(ot_state *st, double *x) {
        double *bs = st->sums.p + 6 * (K + 2);
        slice_sums<double>(st, x, nullptr, nf, K + 1, bs);
        k_slice_shift<double><<<grid2(nf, K + 1), BS, 0, st->stream>>>(nf, bs, 1.0 / nf, x);
    }

    double dot(ot_state *st, const double *a, const double *b) {
        double *out = st->sums.p + 7 * (K + 2);
        const int nblk = std::min(256, std::max(1, ceil_div((int64_t)nphi, BS)));
        k_seg_dot_partial<double><<<dim3(nblk, 1), BS, 0, st->stream>>>(a, b, (int)nphi, st->red.part);
        k_seg_final<<<1, BS, 0, st->stream>>>(st->red.part, nblk, out);
        return st->red.fetch(out, 1)[0];
    }

    // one V-cycle of the Laplacian multigrid, zero-sum per slice
    void prec(ot_state *st, const double *r, double *z) {
        pcg_prec(st, r, z);
        zero_sum(st, z);
    }

    // PCG on S_p x = b (b zero-sum per slice), x = 0 start; returns iterations
    int sp_pcg(ot_state *st, const double *b, double *x, double tol, int maxit) {
        hipStream_t s = st->stream;
        k_fill<double><<<grid1(nphi), BS, 0, s>>>(x, nphi, 0.0);
        k_convert<double, double><<<grid1(nphi), BS, 0, s>>>(b, pr2, nphi);
        const double bn = std::sqrt(std::max(dot(st, pr2, pr2), 0.0));
        if (bn == 0.0) return 0;
        prec(st, pr2, pz2);
        k_convert<double, double><<<grid1(nphi), BS, 0, s>>>(pz2, pp2, nphi);
        double rz = dot(st, pr2, pz2);
        int it = 0;
        for (it = 1; it <= maxit; ++it) {
            sp_apply(st, pp2, pq2);
            const double pq = dot(st, pp2, pq2);
            if (!(pq > 0.0)) break;
            const double alpha = rz / pq;
            k_axpby<double><<<grid1(nphi), BS, 0, s>>>(nphi, alpha, pp2, 1.0, x);
            k_axpby<double><<<grid1(nphi), BS, 0, s>>>(nphi, -alpha, pq2, 1.0, pr2);
            if (std::sqrt(std::max(dot(st, pr2, pr2), 0.0)) <= tol * bn) break;
            prec(st, pr2, pz2);
            const double rz2 = dot(st, pr2, pz2);
            k_axpby<double><<<grid1(nphi), BS, 0, s>>>(nphi, 1.0, pz2, rz2 / rz, pp2);
            rz = rz2;
        }
        return std::min(it, maxit);
    }

    void apply(ot_state *st, const double *rin, double *zout) override {
        hipStream_t s = st->stream;
        const double *f = rin, *g = rin + nphi;
        // t = f + B^T P^T C^-1 g, zero-sum per slice
        k_dscale<double><<<grid1(mrho), BS, 0, s>>>(mrho, cdg, 1, g, vr);
        saddle_phi(st, nullptr, vr, t);
        k_axpby<double><<<grid1(nphi), BS, 0, s>>>(nphi, 1.0, f, 1.0, t);
        zero_sum(st, t);
        st->acc.inner_S_iters += sp_pcg(st, t, xs, st->opt.eps_in_S, st->opt.max_inner);
        zero_sum(st, xs);
        // y = C^-1 (P B x - g)
        pb(st, xs, ub);
        k_axpby<double><<<grid1(mrho), BS, 0, s>>>(mrho, -1.0, g, 1.0, ub);
        k_dscale<double><<<grid1(mrho), BS, 0, s>>>(mrho, cdg, 1, ub, zout + nphi);
        k_convert<double, double><<<grid1(nphi), BS, 0, s>>>(xs, zout, nphi);
        st->acc.prec_applies++;
    }

    // component access of the BB preconditioner: not part of this one
    void schur_apply_d(ot_state *, const double *, double *) override { unsupported(); }
    int schur_solve_d(ot_state *, const double *, double *, double, int) override { unsupported(); return 0; }
    void tri_diagonals_d(ot_state *, double *, double *, double *) override { unsupported(); }
    void tri_solve_d(ot_state *, const double *, double *) override { unsupported(); }
    int laplace_solve_d(ot_state *, const double *, double *, double, int) override { unsupported(); return 0; }
    void vcycle_d(ot_state *, const double *, double *) override { unsupported(); }
    size_t level_data_d(ot_state *, int, int, double *) override { unsupported(); return 0; }
    static void unsupported() {
        throw OtError(OT_EINVAL, "inspection call of the BB preconditioner on a state using the primal-Schur "
                                 "preconditioner");
    }
};

namespace otbb {

// the preconditioner in use: OT_PREC_HYBRID is BB until it switches to SIMPLE
static int active_preconditioner(const ot_state *st) {
    if (st->opt.preconditioner == OT_PREC_HYBRID) return st->hybrid_simple ? OT_PREC_SIMPLE : OT_PREC_BB;
    return st->opt.preconditioner;
}

static void ensure_prec(ot_state *st) {
    const int pc = active_preconditioner(st);
    const bool fp64_only = pc == OT_PREC_SIMPLE || pc == OT_PREC_PRIMAL;
    const int kind = 2 * pc + (fp64_only ? OT_FP64 : st->opt.precision);
    if (st->prec && st->prec_kind == kind) return;
    std::unique_ptr<PrecBase> &slot = st->precs[kind];
    if (!slot) {
        if (pc == OT_PREC_SIMPLE) slot.reset(new SimplePrec());
        else if (pc == OT_PREC_PRIMAL) slot.reset(new PrimalPrec());
        else if (st->opt.precision == OT_MIXED) slot.reset(new BBPrec<float>());
        else slot.reset(new BBPrec<double>());
    }
    st->prec = slot.get();
    st->prec_kind = kind;
    st->lin_valid = false;
}

static void linearize(ot_state *st) {
    ensure_prec(st);
    if (!st->lin_valid) {
        st->prec->setup(st);
        st->lin_valid = true;
    }
}

// ---------------------------------------------------------------------------
// FGMRES on J_P with the BB preconditioner: x = J_P^-1 b (x zero start)
// ---------------------------------------------------------------------------
// Grow a column store of length-N vectors to hold at least `cols` columns
// (capacity doubles, capped at `cap`), keeping the columns already written.
// Without restart the basis can reach 400 columns; growing on demand keeps
// the footprint at what the iteration count actually needs.
static void ensure_cols(ot_state *st, DBuf<double> &B, int cols, int cap) {
    const size_t N = st->N;
    if (B.n >= (size_t)cols * N) return;
    const int have = (int)(B.n / N);
    const int want = std::max(cols, std::min(cap, std::max(16, 2 * have)));
    DBuf<double> nb((size_t)want * N);
    if (B.n) OT_HIP(hipMemcpyAsync(nb.p, B.p, B.n * sizeof(double), hipMemcpyDeviceToDevice, st->stream));
    OT_HIP(hipStreamSynchronize(st->stream));
    B = std::move(nb);
}

// Tightening rule of the outer solve: once FGMRES meets its tolerance, the
// step length of the trial direction is evaluated; while it is below
// alpha_ok (and still grew by 10% since the last check), the tolerance is
// divided by 100, down to tol_floor_abs, and the iteration continues in the
// same Krylov space.  Near the positivity boundary a direction that meets
// eps_out can still be wrong by more than rho in a few cells, which caps
// the step length; the Newton iteration then crawls at steps of 1e-2.
struct TightenRule {
    std::function<double(const double *)> alpha;   // step length of direction x
    double alpha_ok = 0.9;
    double tol_floor_abs = 0.0;
};

static int fgmres(ot_state *st, const double *b, double *x, double tol_abs, int maxit, double *res_out,
                  const TightenRule *tr = nullptr) {
    hipStream_t s = st->stream;
    const size_t N = st->N;
    const int m = std::max(1, std::min(st->opt.restart, maxit));
    ensure_cols(st, st->V, 1, m + 1);
    k_fill<double><<<grid1(N), BS, 0, s>>>(x, N, 0.0);
    double beta = norm2<double>(st, b, N);
    *res_out = beta;
    if (beta <= tol_abs) return 0;
    k_convert<double, double><<<grid1(N), BS, 0, s>>>(b, st->V.p, N);
    Givens G(m);
    int its = 0;
    double res = beta;
    std::vector<double> h(m + 1), hist;
    bool stop = false, first_cycle = true;
    double alpha_prev = -1.0;
    const double beta0 = beta;
    while (its < maxit) {
        k_axpby<double><<<grid1(N), BS, 0, s>>>(N, 0.0, st->V.p, 1.0 / beta, st->V.p);
        G.reset(beta);
        int j = 0;
        for (;;) {
            bool breakdown = false;
            for (; j < m && its < maxit; ++j) {
                ensure_cols(st, st->Z, j + 1, m);
                ensure_cols(st, st->V, j + 2, m + 1);
                double *zj = st->Z.p + (size_t)j * N;
                st->prec->apply(st, st->V.p + (size_t)j * N, zj);
                double *wn = st->V.p + (size_t)(j + 1) * N;
                apply_saddle(st, zj, wn);
                double hn = cgs2<double>(st, st->V.p, N, j + 1, wn, N, h.data());
                for (int i = 0; i <= j; ++i) G.h(i, j) = h[i];
                G.h(j + 1, j) = hn;
                ++its;
                res = G.push(j);
                if (hn > 0) k_axpby<double><<<grid1(N), BS, 0, s>>>(N, 0.0, wn, 1.0 / hn, wn);
                if (st->opt.verbose > 1) fprintf(stderr, "    fgmres it %d res %.3e target %.3e\n", its, res, tol_abs);
                hist.push_back(res);
                // plateau: no halving over the last 40 iterations (after 80) once
                // the residual is already within accept_relres of the initial
                // one, where the step is taken anyway: near a converged Newton
                // iterate the residual meets the rounding floor of the operator
                // well above eps_out |b|, and the cap would only add time
                const bool stalled = !st->no_plateau && its >= 80 && res > 0.5 * hist[its - 41] &&
                                     res <= st->opt.accept_relres * beta0;
                if (res <= tol_abs || hn == 0.0 || stalled) { stop = stalled; breakdown = hn == 0.0; ++j; break; }
            }
            // x = x_cycle_start + Z y; the first cycle starts from x = 0
            std::vector<double> y = G.solve(j);
            OT_HIP(hipMemcpyAsync(st->shift.p, y.data(), j * sizeof(double), hipMemcpyHostToDevice, s));
            k_combine<double, double><<<grid1(N), BS, 0, s>>>(N, st->Z.p, N, j, st->shift.p, first_cycle ? 0.0 : 1.0, x);
            OT_HIP(hipStreamSynchronize(s));
            if (tr && first_cycle && res <= tol_abs && !stop && !breakdown && j < m && its < maxit &&
                tol_abs > tr->tol_floor_abs) {
                const double a = tr->alpha(x);
                if (st->opt.verbose)
                    fprintf(stderr, "    fgmres %d its at tol %.2e: trial step %.3f\n", its, tol_abs / beta0, a);
                if (a < tr->alpha_ok && (alpha_prev < 0.0 || a > 1.1 * alpha_prev)) {
                    alpha_prev = a;
                    tol_abs = std::max(0.01 * tol_abs, tr->tol_floor_abs);
                    st->acc.tightenings++;
                    continue;                       // same Krylov space, tighter target
                }
            }
            break;
        }
        if (res <= tol_abs || its >= maxit || stop) break;
        first_cycle = false;
        // restart with the true residual
        apply_saddle(st, x, st->V.p);
        k_axpby<double><<<grid1(N), BS, 0, s>>>(N, 1.0, b, -1.0, st->V.p);
        beta = norm2<double>(st, st->V.p, N);
        res = beta;
        if (beta <= tol_abs) break;
    }
    *res_out = res;
    return its;
}

// Solve J_s (dphi; drho) = (f; g~) through the projected system and the
// recovery of Sec. 4.4.1-2.  rhs holds (f; g~) on entry (g~ also in gt);
// solution written to sol.  Returns FGMRES iterations; sets last_converged.
// Step length min(1, tau alpha_max) that the trial solution sol of the
// projected system would give (the common rule): drho = P^T drho_hat,
// ds = (h - s drho) / rho, largest step keeping rho and s positive.  Leaves
// the state untouched (scratch: tmpr, ds, sums, reduction buffers).
static double trial_alpha(ot_state *st, const double *sol) {
    const ot_mesh *m = st->mesh;
    hipStream_t s = st->stream;
    const int K = st->K, nc = m->h.nc;
    double *cs = st->sums.p + 6 * (K + 2);
    slice_sums<double>(st, sol + st->nphi, m->ac, nc, K, cs);
    k_convert<double, double><<<grid1(st->mrho), BS, 0, s>>>(sol + st->nphi, st->tmpr.p, st->mrho);
    k_slice_shift<double><<<grid2(nc, K), BS, 0, s>>>(nc, cs, 1.0 / st->area, st->tmpr.p);
    const int nblk = grid1(st->mrho);
    k_ds_ratio<<<nblk, BS, 0, s>>>(st->mrho, st->view(), st->mu, st->tmpr.p, st->ds, st->red.part);
    k_min_final<<<1, BS, 0, s>>>(st->red.part, nblk, st->red.dev);
    k_min_final<<<1, BS, 0, s>>>(st->red.part.p + nblk, nblk, st->red.dev.p + 1);
    const double *am = st->red.fetch(st->red.dev, 2);
    return std::min(1.0, st->opt.frac_to_boundary * std::min(am[0], am[1]));
}

static int solve_newton_system(ot_state *st, double rhs_norm_abs, bool tighten = false) {
    const ot_mesh *m = st->mesh;
    hipStream_t s = st->stream;
    const int K = st->K, nf = m->h.nf, nc = m->h.nc;
    MeshView mv = mesh_view(m);
    StateView sv = st->view();
    // projected right-hand side (f; P g~)
    double *cs = st->sums.p;
    slice_sums<double>(st, st->rhs.p + st->nphi, nullptr, nc, K, cs);
    k_proj_fix<double><<<grid2(nc, K), BS, 0, s>>>(m->ac, nc, cs, st->area, st->rhs.p + st->nphi);
    linearize(st);
    double t0 = now_s();
    double res = 0.0;
    const double tol = st->opt.eps_out * rhs_norm_abs;
    TightenRule rule;
    rule.alpha = [st](const double *x) { return trial_alpha(st, x); };
    rule.tol_floor_abs = st->opt.eps_out_min * rhs_norm_abs;
    const bool use_rule = tighten && st->opt.eps_out_min < st->opt.eps_out;
    int its = fgmres(st, st->rhs, st->sol, tol, st->opt.max_fgmres, &res, use_rule ? &rule : nullptr);
    st->acc.seconds_linear += now_s() - t0;
    st->acc.outer_iters += its;
    st->acc.linear_systems++;
    st->last_iters = its;
    st->last_relres = rhs_norm_abs > 0 ? res / rhs_norm_abs : 0.0;
    st->last_converged = res <= tol;
    st->acc.last_relres = st->last_relres;
    // recovery: drho <- P^T drho; dphi_bar = dphi_hat - area mean; shift
    double *drho = st->sol.p + st->nphi, *dphi = st->sol.p;
    slice_sums<double>(st, drho, m->ac, nc, K, cs);
    k_slice_shift<double><<<grid2(nc, K), BS, 0, s>>>(nc, cs, 1.0 / st->area, drho);
    double *ps = st->sums.p + (K + 2);
    slice_sums<double>(st, dphi, m->a, nf, K + 1, ps);
    k_slice_shift<double><<<grid2(nf, K + 1), BS, 0, s>>>(nf, ps, 1.0 / st->area, dphi);
    dim3 gc = grid2(nc, K);
    k_opB<<<gc, BS, 0, s>>>(mv, sv, dphi, nullptr, nullptr, 0.0, st->tmpr, nullptr);
    k_recover_r<<<gc, BS, 0, s>>>(nc, m->ac, st->gt, st->tmpr, drho, sv, st->red.part);
    double *ls = st->sums.p + 2 * (K + 2);
    k_seg_final<<<K, BS, 0, s>>>(st->red.part, gc.x, ls);
    const double *lam = st->red.fetch(ls, K);
    std::vector<double> shift(K + 1, 0.0);
    for (int k = 1; k <= K; ++k) shift[k] = shift[k - 1] + st->dt * lam[k - 1] / st->area;
    OT_HIP(hipMemcpyAsync(st->shift.p, shift.data(), (K + 1) * sizeof(double), hipMemcpyHostToDevice, s));
    k_add_shift<<<grid2(nf, K + 1), BS, 0, s>>>(nf, st->shift, dphi);
    OT_HIP(hipStreamSynchronize(s));
    return its;
}

// Solve the Newton system held in rhs / gt, and when FGMRES ends above
// accept_relres, once more with the FP64 preconditioner, inner tolerances
// / 10 and the pseudo-Schur cap lifted to the general inner cap (the
// failure policy for the linear solves; the paper reports such failures
// and stops).  strict: retry whenever eps_out was missed.  The right-hand
// side is untouched by a solve, so the retry starts from the same system.
static void solve_with_retry(ot_state *st, double rhs_norm_abs, bool strict = false, bool tighten = false) {
    st->no_plateau = false;
    solve_newton_system(st, rhs_norm_abs, tighten);
    if (st->last_converged || (!strict && st->last_relres <= st->opt.accept_relres)) return;
    const ot_options saved = st->opt;
    const int its1 = st->last_iters;
    const double rr1 = st->last_relres;
    st->opt.precision = OT_FP64;
    st->opt.eps_in_S = 0.1 * saved.eps_in_S;
    st->opt.eps_in_A = 0.1 * saved.eps_in_A;
    st->opt.max_inner_S = std::max(saved.max_inner_S, saved.max_inner);
    linearize(st);
    // the retry runs to the iteration cap: a plateau exit of the first
    // attempt can sit just above accept_relres in the true residual (the
    // plateau test reads the FGMRES estimate), which fails the step
    st->no_plateau = true;
    solve_newton_system(st, rhs_norm_abs, tighten);
    st->no_plateau = false;
    st->acc.linear_systems--;              // one Newton system, two attempts
    if (st->opt.verbose)
        fprintf(stderr, "  retry: fgmres %d relres %.2e -> fgmres %d relres %.2e\n", its1, rr1, st->last_iters,
                st->last_relres);
    st->opt = saved;
    st->lin_valid = false;
}

static void renormalize(ot_state *st) {
    const ot_mesh *m = st->mesh;
    double *mass = st->sums.p;
    slice_sums<double>(st, st->rho.p, m->ac, m->h.nc, st->K, mass);
    k_renorm<<<grid2(m->h.nc, st->K), BS, 0, st->stream>>>(m->h.nc, mass, st->m0, st->rho);
}

// One inexact Newton step (returns OT_OK / OT_ELINSOLVE)
static int newton_step(ot_state *st, double *res_before) {
    const ot_mesh *m = st->mesh;
    hipStream_t s = st->stream;
    const int K = st->K, nc = m->h.nc;
    MeshView mv = mesh_view(m);
    StateView sv = st->view();
    double t0 = now_s();
    const int64_t s0 = st->acc.inner_S_iters, a0 = st->acc.inner_A_iters, p0 = st->acc.prec_applies;
    const double fn = residual(st);
    if (res_before) *res_before = fn;
    // f = -F_phi, g~ = -F_rho + a' F_s / rho
    k_neg_copy<<<grid1(st->nphi), BS, 0, s>>>(st->nphi, st->F, st->rhs);
    dim3 gc = grid2(nc, K);
    k_newton_rhs<<<gc, BS, 0, s>>>(mv, sv, st->F, st->rhs, st->gt, st->red.part, st->nphi, st->mrho);
    st->lin_valid = false;
    double ts = now_s();
    linearize(st);
    OT_HIP(hipStreamSynchronize(s));
    st->acc.seconds_setup += now_s() - ts;
    solve_with_retry(st, fn, false, true);
    if (st->opt.preconditioner == OT_PREC_HYBRID && !st->hybrid_simple) {
        // BB degrades as mu -> 0 (Sec. 4.4.4); SIMPLE stays robust there
        // (Sec. 4.3, Sec. 4.5).  A BB solve that misses eps_out with a
        // direction the positivity line search would cut below
        // hybrid_alpha (an inaccurate direction: a converged one with a short
        // step is the Newton step itself), or that ends above accept_relres,
        // hands this system and the rest of the continuation to SIMPLE.
        const double a = st->last_converged ? 1.0 : trial_alpha(st, st->sol);
        if (a < st->opt.hybrid_alpha || !(st->last_relres <= st->opt.accept_relres)) {
            if (st->opt.verbose)
                fprintf(stderr, "  BB direction: fgmres %d relres %.2e step %.3f -> switching to SIMPLE\n",
                        st->last_iters, st->last_relres, a);
            st->hybrid_simple = true;
            st->acc.linear_systems--;          // the same Newton system, solved again
            linearize(st);
            solve_with_retry(st, fn, false, true);
        }
    }
    if (active_preconditioner(st) == OT_PREC_SIMPLE) st->acc.simple_systems++;
    int rc = OT_OK;
    if (!st->last_converged) {
        st->acc.failures++;
        if (!(st->last_relres <= st->opt.accept_relres)) {                       // state untouched
            if (st->opt.verbose)
                fprintf(stderr, "  mu %.3e |F| %.3e fgmres %d relres %.2e FAILED (%.3fs)\n", st->mu, fn,
                        st->last_iters, st->last_relres, now_s() - t0);
            return OT_ELINSOLVE;
        }
        rc = OT_ELINSOLVE;
    }
    // ds and the step length
    double *drho = st->sol.p + st->nphi;
    int nblk = grid1(st->mrho);
    k_ds_ratio<<<nblk, BS, 0, s>>>(st->mrho, sv, st->mu, drho, st->ds, st->red.part);
    k_min_final<<<1, BS, 0, s>>>(st->red.part, nblk, st->red.dev);
    k_min_final<<<1, BS, 0, s>>>(st->red.part.p + nblk, nblk, st->red.dev.p + 1);
    const double *am = st->red.fetch(st->red.dev, 2);
    if (st->opt.verbose > 2) {
        // where the step length is decided: the cells with the smallest
        // -rho/drho and -s/ds (host copies, diagnostics only)
        std::vector<double> r(st->mrho), dr(st->mrho), sv(st->mrho), dsv(st->mrho);
        OT_HIP(hipMemcpyAsync(r.data(), st->rho.p, st->mrho * 8, hipMemcpyDeviceToHost, s));
        OT_HIP(hipMemcpyAsync(dr.data(), drho, st->mrho * 8, hipMemcpyDeviceToHost, s));
        OT_HIP(hipMemcpyAsync(sv.data(), st->s.p, st->mrho * 8, hipMemcpyDeviceToHost, s));
        OT_HIP(hipMemcpyAsync(dsv.data(), st->ds.p, st->mrho * 8, hipMemcpyDeviceToHost, s));
        OT_HIP(hipStreamSynchronize(s));
        for (int which = 0; which < 2; ++which) {
            const std::vector<double> &x = which ? sv : r, &dx = which ? dsv : dr;
            std::vector<std::pair<double, size_t>> lim;
            for (size_t q = 0; q < st->mrho; ++q)
                if (dx[q] < 0) lim.push_back({-x[q] / dx[q], q});
            std::partial_sort(lim.begin(), lim.begin() + std::min<size_t>(4, lim.size()), lim.end());
            for (size_t t = 0; t < std::min<size_t>(4, lim.size()); ++t) {
                const size_t q = lim[t].second;
                fprintf(stderr, "    limit %s: ratio %.3e at level %zu cell %zu: rho %.3e drho %.3e s %.3e ds %.3e\n",
                        which ? "s" : "rho", lim[t].first, q / nc, q % nc, r[q], dr[q], sv[q], dsv[q]);
            }
        }
    }
    const double tau = st->opt.frac_to_boundary;
    const double a_p = std::min(1.0, tau * am[0]), a_d = std::min(1.0, tau * am[1]);
    // OT_STEP_COMMON: one step for (phi, rho, s); OT_STEP_SPLIT: phi and rho
    // take the largest step keeping rho positive, s its own
    const bool split = st->opt.step_rule == OT_STEP_SPLIT;
    double alpha = std::min(a_p, a_d);
    if (st->opt.neighborhood > 0.0 && !split) {
        // keep (rho, s) in the neighbourhood rho s >= gamma mu of the central path
        k_central_alpha<<<nblk, BS, 0, s>>>(st->mrho, sv, drho, st->ds, st->opt.neighborhood * st->mu, alpha,
                                           st->red.part);
        k_min_final<<<1, BS, 0, s>>>(st->red.part, nblk, st->red.dev);
        alpha = std::min(alpha, st->red.fetch(st->red.dev, 1)[0]);
    }
    const double alpha_p = split ? a_p : alpha, alpha_d = split ? a_d : alpha;
    k_axpy<<<grid1(st->nphi), BS, 0, s>>>(st->nphi, alpha_p, st->sol, st->phi);
    k_axpy<<<grid1(st->mrho), BS, 0, s>>>(st->mrho, alpha_p, drho, st->rho);
    k_axpy<<<grid1(st->mrho), BS, 0, s>>>(st->mrho, alpha_d, st->ds, st->s);
    renormalize(st);
    OT_HIP(hipStreamSynchronize(s));
    st->lin_valid = false;
    st->acc.newton_steps++;
    if (st->opt.verbose) {
        const double np = std::max<int64_t>(1, st->acc.prec_applies - p0);
        fprintf(stderr, "  mu %.3e |F| %.3e fgmres %d relres %.2e inner S %.1f A %.1f alpha %.3f (rho %.3f s %.3f) (%.3fs)\n",
                st->mu, fn, st->last_iters, st->last_relres, (st->acc.inner_S_iters - s0) / np,
                (st->acc.inner_A_iters - a0) / np, alpha, a_p, a_d, now_s() - t0);
    }
    return rc;
}

// outputs: kinetic energy, dual value; optional normalised phi to dst
static void outputs(ot_state *st, double *cost, double *dual) {
    const ot_mesh *m = st->mesh;
    hipStream_t s = st->stream;
    const int K = st->K, nf = m->h.nf, nc = m->h.nc;
    MeshView mv = mesh_view(m);
    StateView sv = st->view();
    dim3 ge = grid2(m->h.ne, K + 1);
    k_ke_partial<<<ge, BS, 0, s>>>(mv, sv, st->red.part);
    double *ke = st->red.seg_final(1, ge.x * ge.y, 0);
    double kev = 0.5 * st->dt * st->red.fetch(ke, 1)[0];
    // D* terms per coarse cell
    double *b = st->tmpN.p;
    const double *pf = st->phi.p, *pl = st->phi.p + (size_t)K * nf;
    k_boundary_terms<<<grid1(nc, 1 << 20), BS, 0, s>>>(mv, sv, pf, pl, b, b + nc, b + 2 * nc, b + 3 * nc);
    std::vector<double> h(4 * (size_t)nc), rin(nc), rf(nc);
    OT_HIP(hipMemcpyAsync(h.data(), b, 4 * nc * sizeof(double), hipMemcpyDeviceToHost, s));
    OT_HIP(hipMemcpyAsync(rin.data(), st->rin.p, nc * sizeof(double), hipMemcpyDeviceToHost, s));
    OT_HIP(hipMemcpyAsync(rf.data(), st->rf.p, nc * sizeof(double), hipMemcpyDeviceToHost, s));
    OT_HIP(hipStreamSynchronize(s));
    double d = 0.0;
    for (int j = 0; j < nc; ++j)
        d += h[nc + j] * rf[j] - h[j] * rin[j] - 0.25 * st->dt * (rin[j] * h[2 * nc + j] + rf[j] * h[3 * nc + j]);
    if (cost) *cost = kev;
    if (dual) *dual = d;
}

static void normalized_phi(ot_state *st, double *dst) {
    const ot_mesh *m = st->mesh;
    const int K = st->K, nf = m->h.nf;
    double *ps = st->sums.p;
    slice_sums<double>(st, st->phi.p, m->a, nf, K + 1, ps);
    const double *h = st->red.fetch(ps, K + 1);
    double tot = 0.0;
    for (int k = 0; k <= K; ++k) tot += h[k];
    const double c = tot / ((K + 1) * st->area);
    k_convert<double, double><<<grid1(st->nphi), BS, 0, st->stream>>>(st->phi, dst, st->nphi);
    k_fill<double><<<1, BS, 0, st->stream>>>(st->shift.p, K + 2, c);
    k_slice_shift<double><<<grid2(nf, K + 1), BS, 0, st->stream>>>(nf, st->shift, 1.0, dst);
    OT_HIP(hipStreamSynchronize(st->stream));
}

}  // namespace otbb

// ===========================================================================
// C ABI
// ===========================================================================
namespace {

template <typename F>
int guard(F &&f) {
    try {
        f();
        return OT_OK;
    } catch (const OtError &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return OT_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return OT_EDEVICE;
    }
}

hipStream_t opt_stream(const ot_options *o) { return o ? (hipStream_t)o->stream : nullptr; }

void copy_in(double *dst, const double *src, size_t n, int mem_kind, hipStream_t s) {
    OT_HIP(hipMemcpyAsync(dst, src, n * sizeof(double),
                          mem_kind == OT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
}
void copy_out(double *dst, const double *src, size_t n, int mem_kind, hipStream_t s) {
    OT_HIP(hipMemcpyAsync(dst, src, n * sizeof(double),
                          mem_kind == OT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
}

void check_options(const ot_options &o) {
    OT_REQUIRE(o.tol > 0 && o.eps_out > 0 && o.eps_in_S > 0 && o.eps_in_A > 0, OT_EINVAL, "tolerances must be > 0");
    OT_REQUIRE(o.mu0 > 0 && o.mu_factor > 0 && o.mu_factor < 1, OT_EINVAL, "bad mu schedule");
    OT_REQUIRE(o.frac_to_boundary > 0 && o.frac_to_boundary < 1, OT_EINVAL, "bad step fraction");
    OT_REQUIRE(o.accept_relres >= 0 && o.accept_relres < 1, OT_EINVAL, "bad accept_relres");
    OT_REQUIRE(o.max_seconds >= 0.0, OT_EINVAL, "max_seconds must be >= 0");
    OT_REQUIRE(o.neighborhood >= 0.0 && o.neighborhood < 1.0, OT_EINVAL, "neighborhood must be in [0, 1)");
    OT_REQUIRE(o.eps_out_min > 0, OT_EINVAL, "eps_out_min must be > 0");
    OT_REQUIRE(o.max_fgmres >= 1 && o.restart >= 1 && o.restart < kMaxBasis && o.max_inner >= 1 && o.max_inner_S >= 1 &&
                   (o.step_rule == OT_STEP_COMMON || o.step_rule == OT_STEP_SPLIT) && o.mu_stop >= 0.0 &&
                   o.max_newton >= 1 && o.inner_restart >= 2 && o.inner_restart < kMaxBasis,
               OT_EINVAL, "bad iteration caps");
    OT_REQUIRE(o.precision == OT_FP64 || o.precision == OT_MIXED, OT_EINVAL, "bad precision");
    OT_REQUIRE(o.preconditioner == OT_PREC_BB || o.preconditioner == OT_PREC_SIMPLE ||
                   o.preconditioner == OT_PREC_HYBRID || o.preconditioner == OT_PREC_PRIMAL,
               OT_EINVAL, "bad preconditioner");
    OT_REQUIRE(o.hybrid_alpha >= 0.0 && o.hybrid_alpha <= 1.0, OT_EINVAL, "hybrid_alpha must be in [0, 1]");
    OT_REQUIRE(o.mem_kind == OT_HOST || o.mem_kind == OT_DEVICE, OT_EINVAL, "bad mem_kind");
}

// host copy of marginals for validation (from host or device memory)
std::vector<double> fetch_vec(const double *p, size_t n, int mem_kind, hipStream_t s) {
    std::vector<double> h(n);
    if (mem_kind == OT_DEVICE) {
        OT_HIP(hipMemcpyAsync(h.data(), p, n * sizeof(double), hipMemcpyDeviceToHost, s));
        OT_HIP(hipStreamSynchronize(s));
    } else {
        std::memcpy(h.data(), p, n * sizeof(double));
    }
    return h;
}

void validate_marginals(const ot_mesh *m, const std::vector<double> &ri, const std::vector<double> &rf) {
    double mi = 0, mf = 0;
    for (int j = 0; j < m->h.nc; ++j) {
        OT_REQUIRE(std::isfinite(ri[j]) && ri[j] >= 0 && std::isfinite(rf[j]) && rf[j] >= 0, OT_ENEG,
                   "marginals must be finite and >= 0");
        mi += m->h.ac[j] * ri[j];
        mf += m->h.ac[j] * rf[j];
    }
    OT_REQUIRE(mi > 0, OT_ENEG, "marginal mass must be > 0");
    OT_REQUIRE(std::fabs(mi - mf) <= 1e-12 * mi, OT_EMASS, "marginals have different mass");
}

ot_state *create_state(const ot_mesh *m, const double *rho_in, const double *rho_f, int K, const ot_options &o) {
    OT_REQUIRE(m && rho_in && rho_f, OT_EINVAL, "null argument");
    OT_REQUIRE(K >= 1, OT_EINVAL, "K must be >= 1");
    check_options(o);
    hipStream_t s = opt_stream(&o);
    auto ri = fetch_vec(rho_in, m->h.nc, o.mem_kind, s);
    auto rf = fetch_vec(rho_f, m->h.nc, o.mem_kind, s);
    validate_marginals(m, ri, rf);
    std::unique_ptr<ot_state> st(new ot_state());
    st->mesh = m;
    st->K = K;
    st->opt = o;
    st->stream = s;
    const int nf = m->h.nf, nc = m->h.nc;
    st->nphi = (size_t)(K + 1) * nf;
    st->mrho = (size_t)K * nc;
    st->N = st->nphi + st->mrho;
    st->dt = 1.0 / (K + 1);
    st->area = m->area;
    st->mu = o.mu0;
    st->m0 = 0.0;
    for (int j = 0; j < nc; ++j) st->m0 += m->h.ac[j] * ri[j];
    st->phi.alloc(st->nphi); st->rho.alloc(st->mrho); st->s.alloc(st->mrho);
    st->rin.upload(ri, s); st->rf.upload(rf, s);
    st->F.alloc(st->nphi + 2 * st->mrho);
    st->rhs.alloc(st->N); st->sol.alloc(st->N); st->gt.alloc(st->mrho);
    st->tmpN.alloc(std::max(st->N, (size_t)8 * nc)); st->tmpr.alloc(st->mrho); st->ds.alloc(st->mrho);
    st->sums.alloc(8 * (K + 2) + 256);
    st->shift.alloc(std::max(K + 2, kMaxBasis + 1));
    size_t np = (size_t)(ceil_div(std::max(std::max(nf, nc), std::max(m->h.ne, 1)), BS) + 1) * (2 * K + 4) +
                (size_t)kMaxBasis * kMultidotBlocks;
    st->red.init(np, std::max<size_t>(2 * kMaxBasis + 1, 8 * (size_t)(K + 2)), s);
    // set-up of the allocation-free entry point on this device
    (void)scratch_on_current_device();
    // start point: phi = 0, rho = m0/|Omega|, s = mu0/rho
    k_fill<double><<<grid1(st->nphi), BS, 0, s>>>(st->phi, st->nphi, 0.0);
    k_fill<double><<<grid1(st->mrho), BS, 0, s>>>(st->rho, st->mrho, st->m0 / st->area);
    k_fill<double><<<grid1(st->mrho), BS, 0, s>>>(st->s, st->mrho, o.mu0 * st->area / st->m0);
    OT_HIP(hipStreamSynchronize(s));
    return st.release();
}

// continuation driver (Sec. 2.4) from the state's current iterate and mu:
// mu, mu f, mu f^2, ... each solved to |F_mu| <= tol by Newton steps, ending
// after the first mu below tol (or at or below mu_stop); returns OT code
int run_ipm(ot_state *st, double tol) {
    const ot_options &o = st->opt;
    double t0 = now_s();
    int rc = OT_OK;
    for (int l = 0; l < 400; ++l) {
        const bool last = st->mu < tol || (o.mu_stop > 0.0 && st->mu <= o.mu_stop * (1.0 + 1e-12));
        const double tl = (last && o.final_tol > 0) ? o.final_tol : tol;
        bool ok = false;
        for (int it = 0; it <= o.max_newton; ++it) {
            double fn = residual(st);
            st->acc.final_residual = fn;
            if (fn <= tl) { ok = true; break; }
            if (it == o.max_newton) break;
            if (o.max_seconds > 0.0 && now_s() - t0 > o.max_seconds) { rc = OT_ETIME; break; }
            int r = newton_step(st, nullptr);
            if (r != OT_OK && !(st->last_relres <= o.accept_relres)) { rc = r; break; }
        }
        st->acc.ip_steps++;
        if (rc != OT_OK) break;
        if (!ok) { rc = OT_ENEWTON; break; }
        if (last) break;
        st->mu *= o.mu_factor;
    }
    st->acc.mu = st->mu;
    st->acc.seconds_total += now_s() - t0;
    return rc;
}

}  // namespace

extern "C" {

void ot_options_default(ot_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-6; o->eps_out = 1e-5; o->eps_in_S = 1e-1; o->eps_in_A = 1e-6;
    o->mu0 = 1.0; o->mu_factor = 0.2; o->frac_to_boundary = 0.99; o->final_tol = 0.0; o->mu_stop = 0.0;
    o->accept_relres = 1e-2;
    o->eps_out_min = 1e-10;
    o->max_fgmres = 400; o->restart = 400; o->max_inner = 200; o->max_newton = 20; o->inner_restart = 30;
    o->max_inner_S = 10;
    o->max_seconds = 0.0;
    o->neighborhood = 0.0;
    o->preconditioner = OT_PREC_HYBRID;
    o->hybrid_alpha = 0.5;
    o->batch_streams = 8;
    o->step_rule = OT_STEP_COMMON;
    o->precision = OT_MIXED; o->mem_kind = OT_HOST; o->verbose = 0; o->stream = nullptr;
}

const char *ot_last_error(void) { return g_last_error.c_str(); }

void ot_abi_sizes(int32_t *options_bytes, int32_t *stats_bytes, int32_t *mesh_desc_bytes) {
    if (options_bytes) *options_bytes = (int32_t)sizeof(ot_options);
    if (stats_bytes) *stats_bytes = (int32_t)sizeof(ot_stats);
    if (mesh_desc_bytes) *mesh_desc_bytes = (int32_t)sizeof(ot_mesh_desc);
}

int ot_kprof_select(int32_t kernel, int32_t elem_bytes) {
    return guard([&] {
        OT_REQUIRE(kernel >= OT_KPROF_NONE && kernel <= OT_KPROF_SADDLE_PHI, OT_EINVAL, "unknown kernel id");
        OT_REQUIRE(elem_bytes == 0 || elem_bytes == 4 || elem_bytes == 8, OT_EINVAL, "elem_bytes must be 0, 4 or 8");
        kprof::Prof &P = kprof::prof();
        std::lock_guard<std::mutex> lk(P.mu);
        for (size_t i = 0; i < P.used; ++i) OT_HIP(hipEventSynchronize(P.pool[i].second));
        P.used = 0;
        P.launches = 0; P.ms = 0.0; P.bytes = 0.0;
        P.width = elem_bytes;
        P.sel = kernel;
    });
}

int ot_kprof_read(int64_t *launches, double *ms, double *bytes) {
    return guard([&] {
        kprof::Prof &P = kprof::prof();
        std::lock_guard<std::mutex> lk(P.mu);
        kprof::drain(P);
        if (launches) *launches = P.launches;
        if (ms) *ms = P.ms;
        if (bytes) *bytes = P.bytes;
    });
}

int ot_mesh_create(const ot_mesh_desc *d, ot_mesh **out) {
    return guard([&] {
        OT_REQUIRE(d && out, OT_EINVAL, "null argument");
        *out = nullptr;
        OT_REQUIRE(d->n_fine > 0 && d->n_coarse > 0 && d->n_overlap >= 0 && d->n_fedge >= 0 && d->n_cedge >= 0,
                   OT_EINVAL, "bad sizes");
        OT_REQUIRE(d->fine_area && d->coarse_area && (d->n_overlap == 0 || (d->ov_fine && d->ov_coarse && d->ov_area)) &&
                       (d->n_fedge == 0 || (d->fe_cell && d->fe_rho && d->fe_len && d->fe_dist && d->fe_lambda)) &&
                       (d->n_cedge == 0 || (d->ce_cell && d->ce_len && d->ce_dist && d->ce_lambda)),
                   OT_EINVAL, "null array in mesh description");
        std::unique_ptr<ot_mesh> m(new ot_mesh());
        MeshHost &h = m->h;
        h.nf = d->n_fine; h.nc = d->n_coarse; h.ne = d->n_fedge; h.nce = d->n_cedge;
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
        mesh_finalize(m.get());
        *out = m.release();
    });
}

int ot_mesh_create_structured(int32_t n, int32_t cartesian, ot_mesh **out) {
    return guard([&] {
        OT_REQUIRE(out, OT_EINVAL, "null argument");
        *out = nullptr;
        OT_REQUIRE(n >= 2 && n <= 16384, OT_EINVAL, "n out of range");
        std::unique_ptr<ot_mesh> m(new ot_mesh());
        structured_desc(n, cartesian != 0, m->h);
        mesh_finalize(m.get());
        *out = m.release();
    });
}

int ot_mesh_create_cartesian3d(int32_t n, ot_mesh **out) {
    return guard([&] {
        OT_REQUIRE(out, OT_EINVAL, "null argument");
        *out = nullptr;
        std::unique_ptr<ot_mesh> m(new ot_mesh());
        cartesian3d_desc(n, m->h);
        mesh_finalize(m.get());
        *out = m.release();
    });
}

void ot_mesh_destroy(ot_mesh *m) { delete m; }

int ot_mesh_sizes(const ot_mesh *m, int32_t *nf, int32_t *nc, int32_t *ne, int32_t *nce) {
    return guard([&] {
        OT_REQUIRE(m, OT_EINVAL, "null mesh");
        if (nf) *nf = m->h.nf;
        if (nc) *nc = m->h.nc;
        if (ne) *ne = m->h.ne;
        if (nce) *nce = m->h.nce;
    });
}

int ot_state_create(const ot_mesh *m, const double *rho_in, const double *rho_f, int32_t K,
                    const ot_options *opt, ot_state **out) {
    return guard([&] {
        OT_REQUIRE(out, OT_EINVAL, "null argument");
        *out = nullptr;
        ot_options o;
        if (opt) o = *opt; else ot_options_default(&o);
        *out = create_state(m, rho_in, rho_f, K, o);
    });
}

void ot_state_destroy(ot_state *st) { delete st; }

int ot_state_sizes(const ot_state *st, int64_t *n_phi, int64_t *m_rho) {
    return guard([&] {
        OT_REQUIRE(st, OT_EINVAL, "null state");
        if (n_phi) *n_phi = (int64_t)st->nphi;
        if (m_rho) *m_rho = (int64_t)st->mrho;
    });
}

int ot_state_set_options(ot_state *st, const ot_options *opt) {
    return guard([&] {
        OT_REQUIRE(st && opt, OT_EINVAL, "null argument");
        check_options(*opt);
        OT_REQUIRE((hipStream_t)opt->stream == st->stream, OT_EINVAL, "stream of a state cannot change");
        const int old_inner = st->opt.inner_restart;
        st->opt = *opt;
        if (old_inner != opt->inner_restart) {     // inner basis size is fixed at allocation
            st->prec = nullptr;
            st->prec_kind = -1;
            st->precs.clear();
        }
        st->lin_valid = false;
    });
}

int ot_state_export(const ot_state *st, double *phi, double *rho, double *s, double *mu) {
    return guard([&] {
        OT_REQUIRE(st, OT_EINVAL, "null state");
        const int mk = st->opt.mem_kind;
        if (phi) copy_out(phi, st->phi, st->nphi, mk, st->stream);
        if (rho) copy_out(rho, st->rho, st->mrho, mk, st->stream);
        if (s) copy_out(s, st->s, st->mrho, mk, st->stream);
        if (mu) *mu = st->mu;
        OT_HIP(hipStreamSynchronize(st->stream));
    });
}

int ot_state_import(ot_state *st, const double *phi, const double *rho, const double *s, double mu) {
    return guard([&] {
        OT_REQUIRE(st && phi && rho && s, OT_EINVAL, "null argument");
        OT_REQUIRE(mu > 0, OT_EINVAL, "mu must be > 0");
        const int mk = st->opt.mem_kind;
        auto hr = fetch_vec(rho, st->mrho, mk, st->stream);
        auto hs = fetch_vec(s, st->mrho, mk, st->stream);
        for (size_t q = 0; q < st->mrho; ++q)
            OT_REQUIRE(std::isfinite(hr[q]) && hr[q] > 0 && std::isfinite(hs[q]) && hs[q] > 0, OT_ENEG,
                       "imported rho and s must be finite and > 0");
        copy_in(st->phi, phi, st->nphi, mk, st->stream);
        copy_in(st->rho, rho, st->mrho, mk, st->stream);
        copy_in(st->s, s, st->mrho, mk, st->stream);
        st->mu = mu;
        st->lin_valid = false;
        st->hybrid_simple = false;
        OT_HIP(hipStreamSynchronize(st->stream));
    });
}

int ot_state_set_mu(ot_state *st, double mu) {
    return guard([&] {
        OT_REQUIRE(st && mu > 0, OT_EINVAL, "bad argument");
        st->mu = mu;
    });
}

int ot_residual(ot_state *st, double *F, double *nrm) {
    return guard([&] {
        OT_REQUIRE(st, OT_EINVAL, "null state");
        double n = residual(st);
        if (nrm) *nrm = n;
        if (F) copy_out(F, st->F, st->nphi + 2 * st->mrho, st->opt.mem_kind, st->stream);
        OT_HIP(hipStreamSynchronize(st->stream));
    });
}

int ot_newton_step(ot_state *st, ot_stats *stats, double *res_norm) {
    int rc = OT_OK;
    int g = guard([&] {
        OT_REQUIRE(st, OT_EINVAL, "null state");
        ot_stats before = st->acc;
        rc = newton_step(st, res_norm);
        if (stats) {
            *stats = st->acc;
            stats->outer_iters -= before.outer_iters;
            stats->inner_S_iters -= before.inner_S_iters;
            stats->inner_A_iters -= before.inner_A_iters;
            stats->prec_applies -= before.prec_applies;
            stats->linear_systems -= before.linear_systems;
            stats->newton_steps -= before.newton_steps;
            stats->failures -= before.failures;
            stats->tightenings -= before.tightenings;
            stats->simple_systems -= before.simple_systems;
        }
        if (rc != OT_OK) set_last_error("FGMRES did not reach eps_out");
    });
    return g != OT_OK ? g : rc;
}

int ot_apply_saddle(ot_state *st, const double *x, double *y) {
    return guard([&] {
        OT_REQUIRE(st && x && y, OT_EINVAL, "null argument");
        const int mk = st->opt.mem_kind;
        copy_in(st->tmpN, x, st->N, mk, st->stream);
        apply_saddle(st, st->tmpN, st->rhs);
        copy_out(y, st->rhs, st->N, mk, st->stream);
        OT_HIP(hipStreamSynchronize(st->stream));
    });
}

int ot_apply_saddle_noalloc(const ot_state *st, const double *x, double *y, void *stream) {
    return guard([&] {
        OT_REQUIRE(st && x && y, OT_EINVAL, "null argument");
        int dev = -1;
        OT_HIP(hipGetDevice(&dev));
        OT_REQUIRE(dev == st->mesh->device, OT_EINVAL, "the state's device must be current");
        const size_t need = saddle_scratch_doubles(st);
        OT_REQUIRE(need <= kNoallocScratch, OT_EINVAL,
                   "problem too large for the library scratch of ot_apply_saddle_noalloc: needs " +
                       std::to_string(need) + " doubles, holds " + std::to_string(kNoallocScratch));
        double *sc = scratch_on_current_device();
        hipStream_t s = stream ? (hipStream_t)stream : st->stream;
        apply_saddle_core(st, x, y, sc, sc + 2 * (size_t)(st->K + 2), s);
        OT_HIP(hipGetLastError());
    });
}

int ot_apply_schur_prec(ot_state *st, const double *r, double *z) {
    return guard([&] {
        OT_REQUIRE(st && r && z, OT_EINVAL, "null argument");
        const int mk = st->opt.mem_kind;
        linearize(st);
        copy_in(st->tmpN, r, st->N, mk, st->stream);
        st->prec->apply(st, st->tmpN, st->rhs);
        copy_out(z, st->rhs, st->N, mk, st->stream);
        OT_HIP(hipStreamSynchronize(st->stream));
    });
}

int ot_outputs(ot_state *st, double *cost, double *dual, double *phi_out) {
    return guard([&] {
        OT_REQUIRE(st, OT_EINVAL, "null state");
        outputs(st, cost, dual);
        if (phi_out) {
            normalized_phi(st, st->tmpN);
            copy_out(phi_out, st->tmpN, st->nphi, st->opt.mem_kind, st->stream);
            OT_HIP(hipStreamSynchronize(st->stream));
        }
    });
}

int ot_solve(const ot_mesh *m, const double *rho_in, const double *rho_f, int32_t K, double tol,
             const ot_options *opt, double *rho_out, double *phi_out, double *cost_out, ot_stats *stats) {
    int rc = OT_OK;
    int g = guard([&] {
        ot_options o;
        if (opt) o = *opt; else ot_options_default(&o);
        if (tol > 0) o.tol = tol;
        std::unique_ptr<ot_state> st(create_state(m, rho_in, rho_f, K, o));
        rc = run_ipm(st.get(), o.tol);
        double cost = 0, dual = 0;
        outputs(st.get(), &cost, &dual);
        st->acc.cost = cost; st->acc.dual = dual; st->acc.gap = cost - dual;
        if (cost_out) *cost_out = cost;
        if (rho_out) copy_out(rho_out, st->rho, st->mrho, o.mem_kind, st->stream);
        if (phi_out) {
            normalized_phi(st.get(), st->tmpN);
            copy_out(phi_out, st->tmpN, st->nphi, o.mem_kind, st->stream);
        }
        OT_HIP(hipStreamSynchronize(st->stream));
        if (stats) *stats = st->acc;
        if (rc == OT_ELINSOLVE) set_last_error("FGMRES failed");
        if (rc == OT_ENEWTON) set_last_error("Newton iteration cap reached");
        if (rc == OT_ETIME) set_last_error("time limit max_seconds reached");
    });
    return g != OT_OK ? g : rc;
}

int ot_state_solve(ot_state *st, double tol, ot_stats *stats) {
    int rc = OT_OK;
    int g = guard([&] {
        OT_REQUIRE(st, OT_EINVAL, "null state");
        const double t = tol > 0 ? tol : st->opt.tol;
        const ot_stats before = st->acc;
        rc = run_ipm(st, t);
        double cost = 0, dual = 0;
        outputs(st, &cost, &dual);
        st->acc.cost = cost; st->acc.dual = dual; st->acc.gap = cost - dual;
        if (stats) {
            *stats = st->acc;
            stats->ip_steps -= before.ip_steps;
            stats->newton_steps -= before.newton_steps;
            stats->linear_systems -= before.linear_systems;
            stats->outer_iters -= before.outer_iters;
            stats->inner_S_iters -= before.inner_S_iters;
            stats->inner_A_iters -= before.inner_A_iters;
            stats->prec_applies -= before.prec_applies;
            stats->failures -= before.failures;
            stats->tightenings -= before.tightenings;
            stats->simple_systems -= before.simple_systems;
            stats->seconds_total -= before.seconds_total;
            stats->seconds_linear -= before.seconds_linear;
            stats->seconds_setup -= before.seconds_setup;
        }
        if (rc == OT_ELINSOLVE) set_last_error("FGMRES failed");
        if (rc == OT_ENEWTON) set_last_error("Newton iteration cap reached");
        if (rc == OT_ETIME) set_last_error("time limit max_seconds reached");
    });
    return g != OT_OK ? g : rc;
}

int ot_solve_batched(int32_t nprob, const ot_mesh *const *meshes, const double *const *rho_in,
                     const double *const *rho_f, const int32_t *K, double tol, const ot_options *opt,
                     double *const *rho_out, double *const *phi_out, double *costs, ot_stats *stats) {
    int rc = OT_OK;
    int g = guard([&] {
        OT_REQUIRE(nprob >= 0 && (nprob == 0 || (meshes && rho_in && rho_f && K)), OT_EINVAL, "null argument");
        ot_options o;
        if (opt) o = *opt; else ot_options_default(&o);
        check_options(o);
        OT_REQUIRE(o.batch_streams >= 0, OT_EINVAL, "batch_streams must be >= 0");
        if (nprob == 0) return;
        int dev = 0;
        OT_HIP(hipGetDevice(&dev));
        // inputs may have been produced on the caller's stream
        OT_HIP(hipStreamSynchronize((hipStream_t)o.stream));
        // Members run concurrently, each on a stream of its own driven by one
        // host thread (the Krylov solvers wait on scalars between launches,
        // so one thread per in-flight member keeps the device fed); each
        // member has its own state and its own convergence.
        const int nw = std::max(1, std::min<int>(nprob, o.batch_streams > 0 ? o.batch_streams : 8));
        std::vector<int> rcs(nprob, OT_OK);
        std::vector<std::string> msgs(nprob);
        std::atomic<int> next{0};
        auto worker = [&]() {
            hipStream_t s = nullptr;
            if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
                for (int p; (p = next++) < nprob;) { rcs[p] = OT_EDEVICE; msgs[p] = "stream creation failed"; }
                return;
            }
            ot_options om = o;
            om.stream = s;
            for (int p; (p = next++) < nprob;) {
                rcs[p] = ot_solve(meshes[p], rho_in[p], rho_f[p], K[p], tol, &om, rho_out ? rho_out[p] : nullptr,
                                  phi_out ? phi_out[p] : nullptr, costs ? costs + p : nullptr,
                                  stats ? stats + p : nullptr);
                if (rcs[p] != OT_OK) msgs[p] = ot_last_error();
            }
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        };
        if (nw == 1) {
            worker();
        } else {
            std::vector<std::thread> pool;
            for (int t = 0; t < nw; ++t) pool.emplace_back(worker);
            for (auto &th : pool) th.join();
        }
        for (int p = 0; p < nprob; ++p)
            if (rcs[p] != OT_OK) {
                rc = rcs[p];
                set_last_error("member " + std::to_string(p) + ": " + msgs[p]);
                break;
            }
    });
    return g != OT_OK ? g : rc;
}

int ot_gradient(ot_state *st, double *g_in, double *g_f) {
    int rc = OT_OK;
    int g = guard([&] {
        OT_REQUIRE(st && g_in && g_f, OT_EINVAL, "null argument");
        const ot_mesh *m = st->mesh;
        hipStream_t s = st->stream;
        const int K = st->K, nf = m->h.nf, nc = m->h.nc;
        MeshView mv = mesh_view(m);
        StateView sv = st->view();
        // adjoint right-hand side (0; dt a' s): projected system + recovery
        k_fill<double><<<grid1(st->nphi), BS, 0, s>>>(st->rhs, st->nphi, 0.0);
        dim3 gc = grid2(nc, K);
        k_grad_rhs<<<gc, BS, 0, s>>>(nc, m->ac, sv, st->gt, st->rhs.p + st->nphi, st->red.part);
        const double nrm = std::sqrt(st->red.fetch(st->red.seg_final(1, gc.x * gc.y), 1)[0]);
        st->lin_valid = false;
        linearize(st);
        solve_with_retry(st, nrm, true);
        if (!st->last_converged) {
            st->acc.failures++;
            rc = OT_ELINSOLVE;
        }
        // corrections, envelope terms, assembly and projection, on the device
        double *b = st->tmpN.p, *gi = b + 6 * (size_t)nc, *gf = b + 7 * (size_t)nc;
        const double *q1 = st->sol.p, *qK = st->sol.p + (size_t)K * nf;
        const double *p1 = st->phi.p, *pK = st->phi.p + (size_t)K * nf;
        k_adjoint_corr<<<grid1(nc, 1 << 20), BS, 0, s>>>(mv, p1, q1, 1.0, st->dt, b);
        k_adjoint_corr<<<grid1(nc, 1 << 20), BS, 0, s>>>(mv, pK, qK, -1.0, st->dt, b + nc);
        k_boundary_terms<<<grid1(nc, 1 << 20), BS, 0, s>>>(mv, sv, p1, pK, b + 2 * nc, b + 3 * nc, b + 4 * nc,
                                                          b + 5 * nc);
        const int nblk = ceil_div(nc, BS);
        k_grad_assemble<<<nblk, BS, 0, s>>>(nc, m->ac, st->dt, b, gi, gf, st->red.part);
        k_seg_final<<<3, BS, 0, s>>>(st->red.part, nblk, st->red.dev);
        k_grad_project<<<nblk, BS, 0, s>>>(nc, m->ac, st->red.dev, gi, gf);
        copy_out(g_in, gi, nc, st->opt.mem_kind, s);
        copy_out(g_f, gf, nc, st->opt.mem_kind, s);
        OT_HIP(hipStreamSynchronize(s));
        st->lin_valid = false;
        if (rc != OT_OK) set_last_error("adjoint FGMRES solve did not reach eps_out (FP64 retry included)");
    });
    return g != OT_OK ? g : rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Inspection entry points (include/otbb_debug.h): host pointers in and out
// ---------------------------------------------------------------------------
extern "C" {

static int dbg_vec(ot_state *st, const double *in, size_t nin, double *out, size_t nout,
                   const std::function<void(const double *, double *)> &f) {
    return guard([&] {
        OT_REQUIRE(st && in && out, OT_EINVAL, "null argument");
        linearize(st);
        OT_HIP(hipMemcpyAsync(st->tmpN.p, in, nin * sizeof(double), hipMemcpyHostToDevice, st->stream));
        f(st->tmpN.p, st->rhs.p);
        OT_HIP(hipMemcpyAsync(out, st->rhs.p, nout * sizeof(double), hipMemcpyDeviceToHost, st->stream));
        OT_HIP(hipStreamSynchronize(st->stream));
    });
}

int otbb_debug_schur_apply(ot_state *st, const double *z, double *out) {
    return dbg_vec(st, z, st ? st->mrho : 0, out, st ? st->mrho : 0,
                   [&](const double *a, double *b) { st->prec->schur_apply_d(st, a, b); });
}

int otbb_debug_set_schur_mg(double omega, int32_t nu, int32_t coarse_its, double alpha) {
    return guard([&] {
        OT_REQUIRE(omega > 0.0 && omega <= 1.0, OT_EINVAL, "omega must be in (0, 1]");
        OT_REQUIRE(nu >= 1 && nu <= 16, OT_EINVAL, "nu must be in [1, 16]");
        OT_REQUIRE(coarse_its >= 1 && coarse_its <= 200, OT_EINVAL, "coarse_its must be in [1, 200]");
        OT_REQUIRE(alpha > 0.0 && alpha <= 3.0, OT_EINVAL, "alpha must be in (0, 3]");
        g_smg.omega = omega; g_smg.nu = nu; g_smg.coarse_its = coarse_its; g_smg.alpha = alpha;
    });
}

int otbb_debug_set_schur_blocking(int32_t elem_bytes, int32_t btilde_levels, int32_t out_levels) {
    return guard([&] {
        const bool reset = btilde_levels < 0 && out_levels < 0;
        OT_REQUIRE(reset || (btilde_levels >= 0 && btilde_levels <= 64 && out_levels >= 0 && out_levels <= 64),
                   OT_EINVAL, "levels per thread must be in [0, 64] (or both negative: autotune)");
        OT_REQUIRE(elem_bytes == 0 || elem_bytes == 4 || elem_bytes == 8, OT_EINVAL, "elem_bytes must be 0, 4 or 8");
        for (int r = 0; r < 2; ++r) {
            if (elem_bytes != 0 && elem_bytes != (r ? 8 : 4)) continue;
            if (reset) {
                g_schur_tb_fixed[r] = false;
                continue;
            }
            g_schur_tb[r][0] = btilde_levels;
            g_schur_tb[r][1] = out_levels;
            g_schur_tb_fixed[r] = true;
        }
    });
}

int otbb_debug_tri_solve(ot_state *st, const double *r, double *x) {
    return dbg_vec(st, r, st ? st->mrho : 0, x, st ? st->mrho : 0,
                   [&](const double *a, double *b) { st->prec->tri_solve_d(st, a, b); });
}

int otbb_debug_schur_solve(ot_state *st, const double *rhs, double *z, double tol, int32_t maxit,
                           int32_t *iters) {
    int its = 0;
    int rc = dbg_vec(st, rhs, st ? st->mrho : 0, z, st ? st->mrho : 0,
                     [&](const double *a, double *b) { its = st->prec->schur_solve_d(st, a, b, tol, maxit); });
    if (iters) *iters = its;
    return rc;
}

int otbb_debug_tri_diagonals(ot_state *st, double *d0, double *dl, double *du) {
    return guard([&] {
        OT_REQUIRE(st && d0 && dl && du, OT_EINVAL, "null argument");
        linearize(st);
        double *b = st->tmpN.p;
        const size_t m = st->mrho;
        OT_REQUIRE(st->tmpN.n >= 3 * m, OT_EINVAL, "internal: scratch too small");
        st->prec->tri_diagonals_d(st, b, b + m, b + 2 * m);
        OT_HIP(hipMemcpyAsync(d0, b, m * sizeof(double), hipMemcpyDeviceToHost, st->stream));
        OT_HIP(hipMemcpyAsync(dl, b + m, m * sizeof(double), hipMemcpyDeviceToHost, st->stream));
        OT_HIP(hipMemcpyAsync(du, b + 2 * m, m * sizeof(double), hipMemcpyDeviceToHost, st->stream));
        OT_HIP(hipStreamSynchronize(st->stream));
    });
}

int otbb_debug_laplace_solve(ot_state *st, const double *b, double *x, double tol, int32_t maxit,
                             int32_t *iters) {
    int its = 0;
    int rc = dbg_vec(st, b, st ? st->nphi : 0, x, st ? st->nphi : 0,
                     [&](const double *a, double *o) { its = st->prec->laplace_solve_d(st, a, o, tol, maxit); });
    if (iters) *iters = its;
    return rc;
}

int otbb_debug_mg_level(ot_state *st, int32_t level, int32_t what, double *out, int64_t *count) {
    return guard([&] {
        OT_REQUIRE(st, OT_EINVAL, "null state");
        linearize(st);
        size_t n = st->prec->level_data_d(st, level, what, nullptr);
        if (count) *count = (int64_t)n;
        if (out) {
            DBuf<double> tmp(n);
            st->prec->level_data_d(st, level, what, tmp.p);
            OT_HIP(hipMemcpyAsync(out, tmp.p, n * sizeof(double), hipMemcpyDeviceToHost, st->stream));
            OT_HIP(hipStreamSynchronize(st->stream));
        }
    });
}

int otbb_debug_vcycle(ot_state *st, const double *b, double *x) {
    return dbg_vec(st, b, st ? st->nphi : 0, x, st ? st->nphi : 0,
                   [&](const double *a, double *o) { st->prec->vcycle_d(st, a, o); });
}

}  // extern "C"
