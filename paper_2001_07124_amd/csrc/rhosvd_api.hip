// Host orchestrator behind the C ABI of include/rhosvd.h: validation,
// workspace planning and the launch sequence of RP-HOSVD (Algorithm 6) and
// R-STHOSVD (Algorithm 8 over Algorithm 1).  Nothing here computes on the
// host; every arithmetic step is a kernel in kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "rhosvd.h"

struct rhosvd_ctx {
    int device;
    int num_cu;
    size_t lds_per_block;
    int kernels;    // RHOSVD_KERNELS_*: which streaming kernel families may run
    // tile parameters of the batched passes, tuned once per context
    int tuned = 0, tune_cmax = 64, tune_tpu = 1;
    float tune_ms = 0.0f;
    void* scratch;  // this device's address of the no-alloc scratch (noalloc.hip)
};


namespace {

thread_local int32_t g_last_hip = 0;

int32_t hip_fail(hipError_t e) {
    g_last_hip = static_cast<int32_t>(e);
    return RHOSVD_EHIP;
}

#define RH_HIP(call)                                  \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_);    \
    } while (0)

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures.
struct Carver {
    unsigned char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<unsigned char*>(b)) {}
    template <typename P>
    P* take(size_t bytes) {
        off = (off + 255) & ~static_cast<size_t>(255);
        P* p = base ? reinterpret_cast<P*>(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

constexpr int kMaxSmallK = 64;    // the QR and EVD kernels keep K x K in LDS / registers
constexpr int kSumsqBlocks = 256;
// Omega streams of RP-HOOI (Algorithm 7): the Gaussian start and the sketches
constexpr uint32_t kTagHooiInit = 5, kTagHooiSketch = 6, kTagRpetCore = 3, kTagKr = 4;
// The single-pass sketch of all modes regenerates Omega rows per tile: it is
// used while that costs at most this many normals per element of X (beyond
// it the per-mode passes, which generate each row once, are faster).
constexpr double kAllModeNormalsPerElement = 4.0;

// One streaming pass, on the first kernel family that takes the shape:
//   COL    contiguous unfolding (L = 1), bf16 matrix cores (kernels_col.hip)
//   WAVE   any view, FP32 data, wave-private blocks (kernels_wave.hip)
//   TILED  anything, FP32 or FP64 data, workgroup tiles (kernels.hip)
enum PassKind { PASS_TILED = 0, PASS_WAVE = 1, PASS_COL = 2, PASS_TRUNC = 3 };

struct Pass {
    int op = 0;
    int kind = PASS_TILED;
    bool dbl = false;
    rh::StreamGeom sg{};
    rh::WGeom wg{};
    rh::ColGeom cg{};
    rh::TruncGeom tg{};               // PASS_TRUNC (batch only): the rotated truncation kernel
    int grid = 0, I_pad = 0, K_pad = 0, K = 0;
    int64_t I = 0;
};

// kernels == RHOSVD_KERNELS_TILED restricts the choice to the workgroup-tiled
// family (every shape it takes gives the same result to rounding).
bool plan_pass(int op, bool dbl, int ct, int64_t L, int64_t I, int64_t T, int K, int num_cu,
               Pass* p, int kernels = RHOSVD_KERNELS_AUTO) {
    p->op = op;
    p->dbl = dbl;
    p->I = I;
    p->K = K;
    const bool any = kernels == RHOSVD_KERNELS_AUTO;
    if (!dbl && any && rh::plan_col(op, ct, L, I, T, K, num_cu, &p->cg)) {
        p->kind = PASS_COL;
        p->grid = p->cg.grid;
        p->I_pad = p->cg.I_pad;
        p->K_pad = p->cg.K_pad;
        return true;
    }
    // the e4m3 sketch exists in the column kernel only; elsewhere bf16
    if (ct == rh::CT_FP8) ct = rh::CT_BF16;
    if (!dbl && any && rh::plan_wave(op, ct, L, I, T, K, num_cu, &p->wg)) {
        p->kind = PASS_WAVE;
        p->grid = p->wg.grid;
        p->I_pad = p->wg.IB * 16;
        p->K_pad = p->wg.NB * 16;
        return true;
    }
    p->kind = PASS_TILED;
    if (!rh::plan_stream(op, dbl ? 8 : 4, L, I, T, K, num_cu, &p->sg)) return false;
    p->grid = p->sg.grid;
    p->I_pad = p->sg.I_pad;
    p->K_pad = p->sg.K_pad;
    return true;
}

hipError_t launch_pass(const Pass& p, const rh::StreamArgs& a, hipStream_t s) {
    if (p.kind == PASS_COL) return rh::launch_col(p.op, p.cg, a, s);
    if (p.kind == PASS_WAVE) return rh::launch_wave(p.op, p.wg, a, s);
    return rh::launch_stream(p.op, p.dbl, p.sg, a, s);
}

struct Problem {
    int N = 0;
    int64_t dims[RHOSVD_MAX_ORDER] = {};
    bool dbl = false;
    size_t elem = 4;
    int algo = 0;
    int ranks[RHOSVD_MAX_ORDER] = {};
    int p = 0, q = 0;
    uint64_t seed = 0;
    int order[RHOSVD_MAX_ORDER] = {};
    int prec = 0;
    int ct_sketch = 0, ct_power = 0, ct_ttm = 0, ct_trunc = 0;
    int kernels = RHOSVD_KERNELS_AUTO;
    bool explicit_error = false;
    bool kr = false;             // structured (Khatri-Rao) sketch
};

struct Step {
    int n;
    int64_t L, I, T, J;
    int K, R;
    bool capped;
    Pass gs, gp, gt, gtr;
    bool trunc_rot = false;       // the rotated truncation on its own kernel
    rh::TruncGeom tg{};
};

struct Plan {
    Problem pr;
    Step st[RHOSVD_MAX_ORDER];
    // RP-HOSVD core chain geometries
    Pass gh[RHOSVD_MAX_ORDER];   // X..  x_n Q_n^T
    Pass gg[RHOSVD_MAX_ORDER];   // Gram of H_(n) (identity TTM)
    Pass gc[RHOSVD_MAX_ORDER];   // H .. x_n M_n^T
    bool any_k_gt_r = false;
    // RP-HOSVD: every sketch from one read of X when the single-pass kernel
    // takes the shape and its Omega work stays small (see plan_allmode_use)
    bool use_allmode = false;
    rh::AllModeArgs am{};
    // RP-HOOI: per mode n the chain X x_{p != n} Q_p^T (one mode-n product
    // per p != n, natural order) and the sketch of its n-unfolding
    Pass hchain[RHOSVD_MAX_ORDER][RHOSVD_MAX_ORDER];
    Pass hsk[RHOSVD_MAX_ORDER];
    // R-PET: the core sketch X x_n Omt_n^T (widths S_n) and the recovery
    // H x_n pinv(Omt_n^T Q_n), each a chain of mode-n products
    int Sn[RHOSVD_MAX_ORDER] = {};
    Pass gp0[RHOSVD_MAX_ORDER];
    Pass gp1[RHOSVD_MAX_ORDER];
    int64_t omt = 0, pst = 0;
    // structured sketch: per step the tables of the other modes in the
    // digit order of the sketched view (its storage order), at offsets
    // kr_off (elements) into one region of kr_elems
    int64_t kr_elems = 0;
    int kr_mode[RHOSVD_MAX_ORDER][RHOSVD_MAX_ORDER - 1] = {};
    int64_t kr_ext[RHOSVD_MAX_ORDER][RHOSVD_MAX_ORDER - 1] = {};
    int64_t kr_off[RHOSVD_MAX_ORDER][RHOSVD_MAX_ORDER - 1] = {};
    // R-STHOSVD in the natural mode order keeps the current tensor with its
    // next mode first: (I_n, ..., I_N, R_1, ..., R_{n-1}).  Every unfolding is
    // then contiguous (L = 1), its columns are in the cyclic order that
    // indexes Omega, and after the last mode the core is back in (R_1, .., R_N).
    bool rotated = false;
    int64_t core_elems = 1;
    // sizes
    size_t part_bytes = 0;
    int max_grid = 1;
    int64_t maxIK = 1, maxKK = 1, maxKR = 1, maxIR = 1, maxB = 1, maxQW = 1;
    int64_t ping = 1, pong = 1;
    int64_t qstore = 0, mstore = 0, ystore = 0;
};

int64_t prod(const int64_t* d, int a, int b) {
    int64_t v = 1;
    for (int m = a; m < b; ++m) v *= d[m];
    return v;
}

int32_t validate(const rhosvd_tensor* x, const rhosvd_params* p, Problem* pr, bool need_data) {
    if (!x || !p) return RHOSVD_EINVAL;
    if (x->order < 2 || x->order > RHOSVD_MAX_ORDER || !x->dims) return RHOSVD_EINVAL;
    if (x->dtype != RHOSVD_F32 && x->dtype != RHOSVD_F64) return RHOSVD_EINVAL;
    if (need_data && !x->data) return RHOSVD_EINVAL;
    if (p->algo != RHOSVD_RP_HOSVD && p->algo != RHOSVD_R_STHOSVD && p->algo != RHOSVD_RP_HOOI &&
        p->algo != RHOSVD_R_PET)
        return RHOSVD_EINVAL;
    if (p->algo == RHOSVD_RP_HOOI && p->oversample != 0) return RHOSVD_EINVAL;
    if (p->algo == RHOSVD_R_PET && p->power_iters != 0) return RHOSVD_EINVAL;
    if (!p->ranks || p->oversample < 0 || p->power_iters < 0 || p->power_iters > 8)
        return RHOSVD_EINVAL;
    if ((p->flags & ~static_cast<uint32_t>(RHOSVD_OPT_EXPLICIT_ERROR | RHOSVD_OPT_KR_SKETCH)) != 0)
        return RHOSVD_EINVAL;
    pr->kr = (p->flags & RHOSVD_OPT_KR_SKETCH) != 0;
    if (pr->kr && p->algo != RHOSVD_R_STHOSVD && p->algo != RHOSVD_RP_HOSVD) return RHOSVD_EINVAL;
    // R-PET's core is recovered from a sketch, not X x_n U_n^T, so the
    // identity E of Section 5.1 does not hold for it: always the explicit one
    pr->explicit_error = (p->flags & RHOSVD_OPT_EXPLICIT_ERROR) != 0 || p->algo == RHOSVD_R_PET;
    pr->N = x->order;
    pr->dbl = x->dtype == RHOSVD_F64;
    pr->elem = pr->dbl ? sizeof(double) : sizeof(float);
    pr->algo = p->algo;
    pr->p = p->oversample;
    pr->q = p->power_iters;
    pr->seed = p->seed;
    pr->prec = p->precision;
    double total = 1.0;
    for (int n = 0; n < pr->N; ++n) {
        if (x->dims[n] < 1) return RHOSVD_EINVAL;
        pr->dims[n] = x->dims[n];
        total *= static_cast<double>(x->dims[n]);
        if (p->ranks[n] < 1 || p->ranks[n] > x->dims[n]) return RHOSVD_EINVAL;
        pr->ranks[n] = p->ranks[n];
    }
    if (total > 4.0e18) return RHOSVD_EINVAL;
    if (p->mode_order) {
        if (p->algo != RHOSVD_R_STHOSVD) return RHOSVD_EINVAL;
        bool seen[RHOSVD_MAX_ORDER] = {};
        for (int s = 0; s < pr->N; ++s) {
            const int n = p->mode_order[s];
            if (n < 0 || n >= pr->N || seen[n]) return RHOSVD_EINVAL;
            seen[n] = true;
            pr->order[s] = n;
        }
    } else {
        for (int s = 0; s < pr->N; ++s) pr->order[s] = s;
    }
    if (p->precision == RHOSVD_PREC_F64) {
        if (!pr->dbl) return RHOSVD_EINVAL;
    } else if (p->precision == RHOSVD_PREC_F32) {
        if (pr->dbl) return RHOSVD_EINVAL;
    } else if (p->precision == RHOSVD_PREC_BF16 || p->precision == RHOSVD_PREC_FP8E4M3) {
        if (pr->dbl) return RHOSVD_EINVAL;
        pr->ct_sketch = p->precision == RHOSVD_PREC_BF16 ? rh::CT_BF16 : rh::CT_FP8;
        pr->ct_power = rh::CT_BF16X3;
        pr->ct_ttm = rh::CT_BF16X3;
        pr->ct_trunc = rh::CT_BF16X3;
    } else {
        return RHOSVD_EINVAL;
    }
    return RHOSVD_OK;
}

void track_stream(Plan* pl, const Pass& g, bool gram) {
    const size_t y = static_cast<size_t>(g.grid) * g.K_pad * g.I_pad * pl->pr.elem;
    const size_t gg = gram ? static_cast<size_t>(g.grid) * g.K_pad * g.K_pad * pl->pr.elem : 0;
    if (y > pl->part_bytes) pl->part_bytes = y;
    if (gg > pl->part_bytes) pl->part_bytes = gg;
    if (g.grid > pl->max_grid) pl->max_grid = g.grid;
}

// The explicit residual reuses the two intermediate buffers (free once the
// core is written) for W_k = G x_1 U_1 ... x_k U_k, k = 1 .. N-1, odd k in
// ping and even k in pong.
void size_resid(Plan* pl) {
    const Problem& pr = pl->pr;
    int64_t d[RHOSVD_MAX_ORDER];
    for (int n = 0; n < pr.N; ++n) d[n] = pr.ranks[n];
    for (int n = 0; n + 1 < pr.N; ++n) {
        d[n] = pr.dims[n];
        const int64_t sz = prod(d, 0, pr.N);
        if (n % 2 == 0) { if (sz > pl->ping) pl->ping = sz; }
        else { if (sz > pl->pong) pl->pong = sz; }
    }
}

// Tables of the structured sketch of step s (mode n) for the current
// extents d: the other modes in the order their indices vary along the
// sketched view's columns (the view's storage order).
void plan_kr(Plan* pl, int s, int n, const int64_t* d, bool rotated, int K) {
    const int N = pl->pr.N;
    int q = 0;
    for (int t = 1; t < N; ++t) {
        const int m = rotated ? (n + t) % N : (t <= n ? t - 1 : t);
        pl->kr_mode[s][q] = m;
        pl->kr_ext[s][q] = d[m];
        pl->kr_off[s][q] = pl->kr_elems;
        pl->kr_elems += d[m] * K;
        ++q;
    }
}

int32_t build_plan(const Problem& pr, int num_cu, Plan* pl) {
    pl->pr = pr;
    const int N = pr.N;
    const int elem = static_cast<int>(pr.elem);
    int64_t d[RHOSVD_MAX_ORDER];
    for (int n = 0; n < N; ++n) d[n] = pr.dims[n];
    if (pr.algo == RHOSVD_R_STHOSVD) {
        pl->rotated = true;
        for (int s = 0; s < N; ++s)
            if (pr.order[s] != s) pl->rotated = false;
        for (int s = 0; s < N; ++s) {
            Step& st = pl->st[s];
            const int n = pr.order[s];
            st.n = n;
            st.L = pl->rotated ? 1 : prod(d, 0, n);
            st.I = d[n];
            st.T = pl->rotated ? prod(d, 0, N) / d[n] : prod(d, n + 1, N);
            st.J = st.L * st.T;
            st.R = pr.ranks[n];
            if (st.R > st.J) return RHOSVD_EINVAL;
            int64_t K = st.R + static_cast<int64_t>(pr.p);
            st.capped = false;
            if (K > st.I) { K = st.I; st.capped = true; }
            if (K > st.J) { K = st.J; st.capped = true; }
            st.K = static_cast<int>(K);
            if (st.K > kMaxSmallK) return RHOSVD_EUNSUPPORTED;
            if (!plan_pass(rh::OP_SKETCH, pr.dbl, pr.ct_sketch, st.L, st.I, st.T, st.K, num_cu, &st.gs, pr.kernels) ||
                !plan_pass(rh::OP_POWER, pr.dbl, pr.ct_power, st.L, st.I, st.T, st.K, num_cu, &st.gp, pr.kernels) ||
                !plan_pass(rh::OP_TTM, pr.dbl, pr.ct_ttm, st.L, st.I, st.T, st.K, num_cu, &st.gt, pr.kernels) ||
                !plan_pass(rh::OP_TTM, pr.dbl, pr.ct_trunc, st.L, st.K, st.T, st.R, num_cu, &st.gtr, pr.kernels))
                return RHOSVD_EUNSUPPORTED;
            track_stream(pl, st.gs, false);
            if (pr.q > 0) track_stream(pl, st.gp, false);
            track_stream(pl, st.gt, true);
            track_stream(pl, st.gtr, false);
            st.trunc_rot = pl->rotated && pr.kernels == RHOSVD_KERNELS_AUTO &&
                           rh::plan_trunc(pr.dbl, st.K, st.T, st.R, num_cu, false, &st.tg);
            const int64_t IK = st.I * st.K;
            if (IK > pl->maxIK) pl->maxIK = IK;
            if (static_cast<int64_t>(st.K) * st.K > pl->maxKK) pl->maxKK = static_cast<int64_t>(st.K) * st.K;
            if (static_cast<int64_t>(st.K) * st.R > pl->maxKR) pl->maxKR = static_cast<int64_t>(st.K) * st.R;
            if (st.I * st.R > pl->maxIR) pl->maxIR = st.I * st.R;
        {
            const int64_t qw = static_cast<int64_t>(rh::evd_qwork_doubles(st.K, st.I));
            if (qw > pl->maxQW) pl->maxQW = qw;
        }
            if (st.K * st.J > pl->maxB) pl->maxB = st.K * st.J;
            if (pr.kr) plan_kr(pl, s, n, d, pl->rotated, st.K);
            d[n] = st.R;
            if (s < N - 1) {
                const int64_t sz = prod(d, 0, N);
                if (s % 2 == 0) { if (sz > pl->ping) pl->ping = sz; }
                else { if (sz > pl->pong) pl->pong = sz; }
            }
        }
        pl->core_elems = prod(d, 0, N);
        size_resid(pl);
        return RHOSVD_OK;
    }
    // RP-HOSVD: every sketch reads X
    for (int n = 0; n < N; ++n) {
        Step& st = pl->st[n];
        st.n = n;
        st.L = prod(d, 0, n);
        st.I = d[n];
        st.T = prod(d, n + 1, N);
        st.J = st.L * st.T;
        st.R = pr.ranks[n];
        if (st.R > st.J) return RHOSVD_EINVAL;
        int64_t K = st.R + static_cast<int64_t>(pr.p);
        st.capped = false;
        if (K > st.I) { K = st.I; st.capped = true; }
        if (K > st.J) { K = st.J; st.capped = true; }
        st.K = static_cast<int>(K);
        if (st.K > kMaxSmallK) return RHOSVD_EUNSUPPORTED;
        if (st.K > st.R) pl->any_k_gt_r = true;
        if (!plan_pass(rh::OP_SKETCH, pr.dbl, pr.ct_sketch, st.L, st.I, st.T, st.K, num_cu, &st.gs, pr.kernels) ||
            !plan_pass(rh::OP_POWER, pr.dbl, pr.ct_power, st.L, st.I, st.T, st.K, num_cu, &st.gp, pr.kernels))
            return RHOSVD_EUNSUPPORTED;
        track_stream(pl, st.gs, false);
        if (pr.q > 0) track_stream(pl, st.gp, false);
        const int64_t IK = st.I * st.K;
        if (IK > pl->maxIK) pl->maxIK = IK;
        if (static_cast<int64_t>(st.K) * st.K > pl->maxKK) pl->maxKK = static_cast<int64_t>(st.K) * st.K;
        if (static_cast<int64_t>(st.K) * st.R > pl->maxKR) pl->maxKR = static_cast<int64_t>(st.K) * st.R;
        if (st.I * st.R > pl->maxIR) pl->maxIR = st.I * st.R;
        {
            const int64_t qw = static_cast<int64_t>(rh::evd_qwork_doubles(st.K, st.I));
            if (qw > pl->maxQW) pl->maxQW = qw;
        }
        pl->qstore += IK;
        pl->mstore += static_cast<int64_t>(st.K) * st.R;
        if (pr.kr) plan_kr(pl, n, n, d, false, st.K);
    }
    if (pr.algo == RHOSVD_RP_HOOI) {
        // chains X x_{p != n} Q_p^T and the sketches of their n-unfoldings
        for (int n = 0; n < N; ++n) {
            int64_t e[RHOSVD_MAX_ORDER];
            for (int m = 0; m < N; ++m) e[m] = d[m];
            for (int q = 0; q < N; ++q) {
                if (q == n) continue;
                if (!plan_pass(rh::OP_TTM, pr.dbl, pr.ct_ttm, prod(e, 0, q), e[q], prod(e, q + 1, N),
                               pr.ranks[q], num_cu, &pl->hchain[n][q], pr.kernels))
                    return RHOSVD_EUNSUPPORTED;
                track_stream(pl, pl->hchain[n][q], false);
                e[q] = pr.ranks[q];
                const int64_t sz = prod(e, 0, N);
                if (sz > pl->ping) pl->ping = sz;
                if (sz > pl->pong) pl->pong = sz;
            }
            const int64_t Ln = prod(e, 0, n), Tn = prod(e, n + 1, N);
            if (pr.ranks[n] > Ln * Tn) return RHOSVD_EINVAL;
            if (!plan_pass(rh::OP_SKETCH, pr.dbl, pr.ct_sketch, Ln, e[n], Tn, pr.ranks[n], num_cu,
                           &pl->hsk[n], pr.kernels))
                return RHOSVD_EUNSUPPORTED;
            track_stream(pl, pl->hsk[n], false);
        }
    } else {
        int Ks[RHOSVD_MAX_ORDER];
        for (int n = 0; n < N; ++n) Ks[n] = pl->st[n].K;
        if (pr.kernels == RHOSVD_KERNELS_AUTO && !pr.kr &&
            rh::plan_allmode(N, pr.dims, Ks, num_cu, elem, &pl->am)) {
            // Omega normals generated per element of X: sum_n K_n / b_n
            double per_elem = 0.0;
            for (int n = 0; n < N; ++n) per_elem += static_cast<double>(Ks[n]) / pl->am.b[n];
            if (per_elem <= kAllModeNormalsPerElement) {
                pl->use_allmode = true;
                const size_t pb = static_cast<size_t>(pl->am.grid) * pl->am.S * pr.elem;
                if (pb > pl->part_bytes) pl->part_bytes = pb;
                if (pl->am.grid > pl->max_grid) pl->max_grid = pl->am.grid;
                pl->ystore = pl->am.S;
            }
        }
    }
    // core chain H = X x_1 Q_1^T ... x_N Q_N^T (R-PET: the core sketch and
    // its recovery), then G = H x_n M_n^T
    int64_t buf = 1;
    if (pr.algo == RHOSVD_R_PET) {
        for (int n = 0; n < N; ++n) {
            const Step& st = pl->st[n];
            pl->Sn[n] = static_cast<int>(std::min<int64_t>(2 * static_cast<int64_t>(st.K) + 1, st.I));
            if (pl->Sn[n] < st.K) return RHOSVD_EUNSUPPORTED;
            pl->omt += st.I * pl->Sn[n];
            pl->pst += static_cast<int64_t>(pl->Sn[n]) * st.K;
        }
        for (int n = 0; n < N; ++n) {
            const int64_t L = prod(d, 0, n), T = prod(d, n + 1, N);
            if (!plan_pass(rh::OP_TTM, pr.dbl, pr.ct_ttm, L, d[n], T, pl->Sn[n], num_cu, &pl->gp0[n], pr.kernels))
                return RHOSVD_EUNSUPPORTED;
            track_stream(pl, pl->gp0[n], false);
            d[n] = pl->Sn[n];
            const int64_t sz = prod(d, 0, N);
            if (sz > buf) buf = sz;
        }
        for (int n = 0; n < N; ++n) {
            const int64_t L = prod(d, 0, n), T = prod(d, n + 1, N);
            if (!plan_pass(rh::OP_TTM, pr.dbl, pr.ct_ttm, L, d[n], T, pl->st[n].K, num_cu, &pl->gp1[n], pr.kernels))
                return RHOSVD_EUNSUPPORTED;
            track_stream(pl, pl->gp1[n], false);
            d[n] = pl->st[n].K;
            const int64_t sz = prod(d, 0, N);
            if (sz > buf) buf = sz;
        }
    }
    for (int n = 0; n < N && pr.algo != RHOSVD_R_PET; ++n) {
        const int64_t L = prod(d, 0, n), T = prod(d, n + 1, N);
        if (!plan_pass(rh::OP_TTM, pr.dbl, pr.ct_ttm, L, d[n], T, pl->st[n].K, num_cu, &pl->gh[n], pr.kernels))
            return RHOSVD_EUNSUPPORTED;
        track_stream(pl, pl->gh[n], false);
        d[n] = pl->st[n].K;
        const int64_t sz = prod(d, 0, N);
        if (sz > buf) buf = sz;
    }
    for (int n = 0; n < N; ++n) {
        const int64_t L = prod(d, 0, n), T = prod(d, n + 1, N);
        if (!plan_pass(rh::OP_TTM, pr.dbl, pr.ct_ttm, L, d[n], T, d[n], num_cu, &pl->gg[n], pr.kernels))
            return RHOSVD_EUNSUPPORTED;
        track_stream(pl, pl->gg[n], true);
    }
    for (int n = 0; n < N; ++n) {
        const int64_t L = prod(d, 0, n), T = prod(d, n + 1, N);
        if (!plan_pass(rh::OP_TTM, pr.dbl, pr.ct_trunc, L, d[n], T, pl->st[n].R, num_cu, &pl->gc[n], pr.kernels))
            return RHOSVD_EUNSUPPORTED;
        track_stream(pl, pl->gc[n], false);
        d[n] = pl->st[n].R;
        const int64_t sz = prod(d, 0, N);
        if (sz > buf) buf = sz;
    }
    pl->ping = std::max(pl->ping, buf);
    pl->pong = std::max(pl->pong, buf);
    pl->core_elems = prod(d, 0, N);
    size_resid(pl);
    return RHOSVD_OK;
}

struct Buffers {
    rhosvd_report* rep;
    void* part;
    double* part_ss;
    double* y;
    double* q64;   // 2 maxIK doubles (q64 + work)
    void* qT;
    double* C;
    void* M;
    double* u64;
    void* B;
    void* ping;
    void* pong;
    void* qstore;
    void* mstore;
    double* ystore;
    int* gate;
    double* part_resid;
    void* omt;     // R-PET: Omt_n, I_n x S_n each
    void* pst;     // R-PET: pinv(Omt_n^T Q_n)^T, S_n x K_n each
    void* krtab;   // structured sketch tables
};

size_t carve(const Plan& pl, void* ws, Buffers* b) {
    Carver cv(ws);
    const size_t e = pl.pr.elem;
    b->rep = cv.take<rhosvd_report>(sizeof(rhosvd_report));
    b->part = cv.take<void>(pl.part_bytes);
    const int ssn = pl.max_grid > kSumsqBlocks ? pl.max_grid : kSumsqBlocks;
    b->part_ss = cv.take<double>(ssn * sizeof(double));
    b->y = cv.take<double>(pl.maxIK * sizeof(double));
    b->q64 = cv.take<double>(2 * pl.maxIK * sizeof(double));
    b->qT = cv.take<void>(pl.maxIK * e);
    b->C = cv.take<double>(pl.maxKK * sizeof(double));
    b->M = cv.take<void>(pl.maxKR * e);
    b->u64 = cv.take<double>(pl.maxQW * sizeof(double));
    if (pl.pr.algo == RHOSVD_R_STHOSVD) {
        b->B = cv.take<void>(pl.maxB * e);
        b->qstore = nullptr;
        b->mstore = nullptr;
        b->ystore = nullptr;
    } else {
        b->B = nullptr;
        b->qstore = cv.take<void>(pl.qstore * e);
        b->ystore = pl.ystore ? cv.take<double>(pl.ystore * sizeof(double)) : nullptr;
        b->mstore = cv.take<void>(pl.mstore * e);
    }
    b->ping = cv.take<void>(pl.ping * e);
    b->pong = cv.take<void>(pl.pong * e);
    b->gate = cv.take<int>(sizeof(int));
    b->part_resid = cv.take<double>(rh::kResidGrid * sizeof(double));
    b->omt = pl.omt ? cv.take<void>(pl.omt * e) : nullptr;
    b->pst = pl.pst ? cv.take<void>(pl.pst * e) : nullptr;
    b->krtab = pl.kr_elems ? cv.take<void>(pl.kr_elems * e) : nullptr;
    return cv.off + 256;
}

void* at(void* base, int64_t elems, size_t elem) {
    return static_cast<unsigned char*>(base) + static_cast<size_t>(elems) * elem;
}

// The structured sketch's arguments for step s (nq = 0: Gaussian stream).
rh::KrArgs kr_args(const Plan& pl, const Buffers& b, int s, int K, int64_t J) {
    rh::KrArgs k{};
    if (!pl.pr.kr) return k;
    k.nq = pl.pr.N - 1;
    k.K = K;
    k.J = J;
    for (int q = 0; q < k.nq; ++q) {
        k.tab[q] = at(b.krtab, pl.kr_off[s][q], pl.pr.elem);
        k.ext[q] = static_cast<int>(pl.kr_ext[s][q]);
    }
    return k;
}

// Fill the tables of steps [s0, s1) (mode of step s: modes[s]), chunked by
// the launch's descriptor limit.
int32_t fill_kr(const Plan& pl, const Buffers& b, int s0, int s1, const int* modes, const int* Ks,
                hipStream_t s) {
    if (!pl.pr.kr) return RHOSVD_OK;
    const int N = pl.pr.N;
    rh::KrFill f{};
    f.seed = pl.pr.seed;
    f.tag = kTagKr;
    for (int st = s0; st < s1; ++st) {
        for (int q = 0; q < N - 1; ++q) {
            rh::KrFill::Table& t = f.t[f.count++];
            t.out = at(b.krtab, pl.kr_off[st][q], pl.pr.elem);
            t.J = pl.kr_ext[st][q];
            t.K = Ks[st];
            t.word = static_cast<uint32_t>(modes[st] * N + pl.kr_mode[st][q]);
            if (f.count == rh::KrFill::kMax) {
                RH_HIP(rh::launch_kr_fill(pl.pr.dbl, f, s));
                f.count = 0;
            }
        }
    }
    if (f.count) RH_HIP(rh::launch_kr_fill(pl.pr.dbl, f, s));
    return RHOSVD_OK;
}

// q fused power steps Y = S_(n) (S_(n)^T Q), each followed by the QR
// (Algorithm 1 step 2 with the stabilising QR between applications).
int32_t power_steps(const Plan& pl, const Buffers& b, const void* src, const Pass& gp, void* q_out,
                    hipStream_t s) {
    const bool dbl = pl.pr.dbl;
    for (int it = 0; it < pl.pr.q; ++it) {
        rh::StreamArgs pa{};
        pa.src = src;
        pa.mat = q_out;
        pa.part_y = b.part;
        RH_HIP(launch_pass(gp, pa, s));
        RH_HIP(rh::launch_reduce_y(dbl, b.part, gp.grid, static_cast<int>(gp.I), gp.K, gp.I_pad,
                                   gp.K_pad, b.y, s));
        RH_HIP(rh::launch_cqr(b.y, gp.I, gp.K, dbl, q_out, b.q64, &b.rep->flags, s));
    }
    return RHOSVD_OK;
}

// Y = S_(n) Omega, then Q and the power steps.
int32_t sketch_and_orthonormalize(const Plan& pl, const Buffers& b, const void* src,
                                  const Pass& gs, const Pass& gp, int mode,
                                  uint32_t tag, double* norm_dst, void* q_out, hipStream_t s,
                                  const rh::KrArgs& kr = rh::KrArgs{}) {
    const bool want_norm = norm_dst != nullptr;
    const bool dbl = pl.pr.dbl;
    rh::StreamArgs a{};
    a.src = src;
    a.part_y = b.part;
    a.part_ss = want_norm ? b.part_ss : nullptr;
    a.seed = pl.pr.seed;
    a.mode = static_cast<uint32_t>(mode);
    a.tag = tag;
    a.kr = kr;
    RH_HIP(launch_pass(gs, a, s));
    RH_HIP(rh::launch_reduce_y(dbl, b.part, gs.grid, static_cast<int>(gs.I), gs.K, gs.I_pad,
                               gs.K_pad, b.y, s));
    if (want_norm) RH_HIP(rh::launch_reduce_ss(b.part_ss, gs.grid, norm_dst, s));
    RH_HIP(rh::launch_cqr(b.y, gs.I, gs.K, dbl, q_out, b.q64, &b.rep->flags, s));
    return power_steps(pl, b, src, gp, q_out, s);
}

int32_t ttm(const Plan& pl, const Pass& g, const void* src, const void* mat, void* out,
            void* part_g, hipStream_t s, int out_t = 0) {
    rh::StreamArgs a{};
    a.src = src;
    a.mat = mat;
    a.out = out;
    a.part_g = part_g;
    a.out_t = out_t;
    RH_HIP(launch_pass(g, a, s));
    (void)pl;
    return RHOSVD_OK;
}

int32_t run_r_sthosvd(const Plan& pl, const Buffers& b, const void* x, const rhosvd_output* out,
                      hipStream_t s) {
    const bool dbl = pl.pr.dbl;
    const size_t e = pl.pr.elem;
    const int N = pl.pr.N;
    const void* src = x;
    if (pl.pr.kr) {
        int modes[RHOSVD_MAX_ORDER], Ks[RHOSVD_MAX_ORDER];
        for (int si = 0; si < N; ++si) {
            modes[si] = pl.st[si].n;
            Ks[si] = pl.st[si].K;
        }
        const int32_t rc = fill_kr(pl, b, 0, N, modes, Ks, s);
        if (rc != RHOSVD_OK) return rc;
    }
    for (int si = 0; si < N; ++si) {
        const Step& st = pl.st[si];
        int32_t rc = sketch_and_orthonormalize(pl, b, src, st.gs, st.gp, st.n, 2u,
                                               si == 0 ? &b.rep->norm_x2 : nullptr, b.qT, s,
                                               kr_args(pl, b, si, st.K, st.J));
        if (rc != RHOSVD_OK) return rc;
        // B = Q^T S_(n), folded, and C = B B^T
        rc = ttm(pl, st.gt, src, b.qT, b.B, b.part, s);
        if (rc != RHOSVD_OK) return rc;
        RH_HIP(rh::launch_gram_reduce(dbl, b.part, st.gt.grid, st.K, st.gt.K_pad, b.C, s));
        RH_HIP(rh::launch_evd_factor(dbl, b.C, st.K, &b.rep->flags, b.qT, st.I, st.R, 1,
                                     out->factors[st.n], b.M, &b.rep->sigma[st.n][0], b.u64, s));
        void* dst = (si == N - 1) ? out->core : ((si % 2 == 0) ? b.ping : b.pong);
        if (st.trunc_rot) {
            RH_HIP(rh::launch_trunc(dbl, st.tg, b.B, b.M, dst, s));
        } else {
            rc = ttm(pl, st.gtr, b.B, b.M, dst, nullptr, s, pl.rotated ? 1 : 0);
            if (rc != RHOSVD_OK) return rc;
        }
        src = dst;
    }
    (void)e;
    return RHOSVD_OK;
}

int32_t run_rp_hosvd(const Plan& pl, const Buffers& b, const void* x, const rhosvd_output* out,
                     hipStream_t s) {
    const bool dbl = pl.pr.dbl;
    const size_t e = pl.pr.elem;
    const int N = pl.pr.N;
    int64_t qoff[RHOSVD_MAX_ORDER], moff[RHOSVD_MAX_ORDER];
    int64_t qo = 0, mo = 0;
    for (int n = 0; n < N; ++n) {
        qoff[n] = qo;
        moff[n] = mo;
        qo += pl.st[n].I * pl.st[n].K;
        mo += static_cast<int64_t>(pl.st[n].K) * pl.st[n].R;
    }
    if (pl.pr.algo == RHOSVD_RP_HOOI) {
        // Algorithm 7: ||X||^2, the orthonormalised Gaussian start, then per
        // sweep s and mode n: S = X x_{p != n} Q_p^T, W = S_(n) Omega (the
        // stream of mode word s N + n), Q_n = QR(W)
        RH_HIP(rh::launch_sumsq(dbl, x, prod(pl.pr.dims, 0, N), b.part_ss, kSumsqBlocks, s));
        RH_HIP(rh::launch_reduce_ss(b.part_ss, kSumsqBlocks, &b.rep->norm_x2, s));
        for (int n = 0; n < N; ++n) {
            const Step& st = pl.st[n];
            RH_HIP(rh::launch_omega_fill(true, pl.pr.seed, n, kTagHooiInit, st.I, st.K, b.y, s));
            RH_HIP(rh::launch_cqr(b.y, st.I, st.K, dbl, at(b.qstore, qoff[n], e), b.q64,
                                  &b.rep->flags, s));
        }
        void* hb[2] = {b.ping, b.pong};
        for (int sw = 0; sw < pl.pr.q; ++sw) {
            for (int n = 0; n < N; ++n) {
                const void* cur = x;
                int k = 0;
                for (int q = 0; q < N; ++q) {
                    if (q == n) continue;
                    const int32_t rc = ttm(pl, pl.hchain[n][q], cur, at(b.qstore, qoff[q], e), hb[k & 1],
                                           nullptr, s);
                    if (rc != RHOSVD_OK) return rc;
                    cur = hb[k & 1];
                    ++k;
                }
                const Step& st = pl.st[n];
                const Pass& gs = pl.hsk[n];
                rh::StreamArgs a{};
                a.src = cur;
                a.part_y = b.part;
                a.seed = pl.pr.seed;
                a.mode = static_cast<uint32_t>(sw * N + n);
                a.tag = kTagHooiSketch;
                RH_HIP(launch_pass(gs, a, s));
                RH_HIP(rh::launch_reduce_y(dbl, b.part, gs.grid, static_cast<int>(gs.I), gs.K,
                                           gs.I_pad, gs.K_pad, b.y, s));
                RH_HIP(rh::launch_cqr(b.y, st.I, st.K, dbl, at(b.qstore, qoff[n], e), b.q64,
                                      &b.rep->flags, s));
            }
        }
    } else if (pl.use_allmode) {
        // every Y_n from one read of X, then per mode the QR and power steps
        rh::AllModeArgs am = pl.am;
        am.x = x;
        am.part = b.part;
        am.part_ss = b.part_ss;
        am.seed = pl.pr.seed;
        am.tag = 1u;
        RH_HIP(rh::launch_allmode(dbl, am, s));
        RH_HIP(rh::launch_allmode_reduce(dbl, am, b.ystore, s));
        RH_HIP(rh::launch_reduce_ss(b.part_ss, am.grid, &b.rep->norm_x2, s));
        for (int n = 0; n < N; ++n) {
            const Step& st = pl.st[n];
            void* qn = at(b.qstore, qoff[n], e);
            RH_HIP(rh::launch_cqr(b.ystore + am.yoff[n], st.I, st.K, dbl, qn, b.q64, &b.rep->flags, s));
            const int32_t rc = power_steps(pl, b, x, st.gp, qn, s);
            if (rc != RHOSVD_OK) return rc;
        }
    } else {
        if (pl.pr.kr) {
            int modes[RHOSVD_MAX_ORDER], Ks[RHOSVD_MAX_ORDER];
            for (int n = 0; n < N; ++n) {
                modes[n] = n;
                Ks[n] = pl.st[n].K;
            }
            const int32_t rc = fill_kr(pl, b, 0, N, modes, Ks, s);
            if (rc != RHOSVD_OK) return rc;
        }
        for (int n = 0; n < N; ++n) {
            const Step& st = pl.st[n];
            const int32_t rc = sketch_and_orthonormalize(pl, b, x, st.gs, st.gp, n, 1u,
                                                         n == 0 ? &b.rep->norm_x2 : nullptr,
                                                         at(b.qstore, qoff[n], e), s,
                                                         kr_args(pl, b, n, st.K, st.J));
            if (rc != RHOSVD_OK) return rc;
        }
    }
    // H = X x_1 Q_1^T ... x_N Q_N^T; R-PET: the core sketch
    // X x_1 Omt_1^T ... x_N Omt_N^T, then H x_n pinv(Omt_n^T Q_n) for all n
    const void* src = x;
    void* bufs[2] = {b.ping, b.pong};
    int cur = 0;
    if (pl.pr.algo == RHOSVD_R_PET) {
        int64_t oo = 0, po = 0;
        int64_t ooff[RHOSVD_MAX_ORDER], poff[RHOSVD_MAX_ORDER];
        for (int n = 0; n < N; ++n) {
            const Step& st = pl.st[n];
            ooff[n] = oo;
            poff[n] = po;
            oo += st.I * pl.Sn[n];
            po += static_cast<int64_t>(pl.Sn[n]) * st.K;
            RH_HIP(rh::launch_omega_fill(dbl, pl.pr.seed, n, kTagRpetCore, st.I, pl.Sn[n],
                                         at(b.omt, ooff[n], e), s));
            RH_HIP(rh::launch_lsq_pinv(dbl, at(b.omt, ooff[n], e), at(b.qstore, qoff[n], e),
                                       static_cast<int>(st.I), pl.Sn[n], st.K, at(b.pst, poff[n], e),
                                       &b.rep->flags, s));
        }
        for (int n = 0; n < N; ++n) {
            const int32_t rc = ttm(pl, pl.gp0[n], src, at(b.omt, ooff[n], e), bufs[cur], nullptr, s);
            if (rc != RHOSVD_OK) return rc;
            src = bufs[cur];
            cur ^= 1;
        }
        for (int n = 0; n < N; ++n) {
            const int32_t rc = ttm(pl, pl.gp1[n], src, at(b.pst, poff[n], e), bufs[cur], nullptr, s);
            if (rc != RHOSVD_OK) return rc;
            src = bufs[cur];
            cur ^= 1;
        }
    } else {
        for (int n = 0; n < N; ++n) {
            const int32_t rc = ttm(pl, pl.gh[n], src, at(b.qstore, qoff[n], e), bufs[cur], nullptr, s);
            if (rc != RHOSVD_OK) return rc;
            src = bufs[cur];
            cur ^= 1;
        }
    }
    const void* H = src;
    void* scratch = bufs[cur];
    // small THOSVD of H: Gram of each unfolding, EVD, factors
    for (int n = 0; n < N; ++n) {
        const Step& st = pl.st[n];
        int32_t rc = ttm(pl, pl.gg[n], H, nullptr, scratch, b.part, s);
        if (rc != RHOSVD_OK) return rc;
        RH_HIP(rh::launch_gram_reduce(dbl, b.part, pl.gg[n].grid, st.K, pl.gg[n].K_pad, b.C, s));
        RH_HIP(rh::launch_evd_factor(dbl, b.C, st.K, &b.rep->flags, at(b.qstore, qoff[n], e),
                                     st.I, st.R, pl.any_k_gt_r ? 1 : 0, out->factors[n],
                                     at(b.mstore, moff[n], e), &b.rep->sigma[n][0], b.u64, s));
    }
    // G = H x_n M_n^T
    src = H;
    for (int n = 0; n < N; ++n) {
        void* dst = (n == N - 1) ? out->core : scratch;
        const int32_t rc = ttm(pl, pl.gc[n], src, at(b.mstore, moff[n], e), dst, nullptr, s);
        if (rc != RHOSVD_OK) return rc;
        // alternate: the buffer just read becomes the next scratch
        void* was = const_cast<void*>(src);
        src = dst;
        scratch = was;
    }
    return RHOSVD_OK;
}

// Explicit residual (Section 8, eq. Relativeerror) on the device: the gate,
// then W = G x_1 U_1 ... x_{N-1} U_{N-1} by expanding mode products, then one
// pass over X against W and U_N.  Every launch is skipped on the device
// unless the gate opened.
int32_t run_residual(const Plan& pl, const Buffers& b, const void* x, const rhosvd_output* out,
                     hipStream_t s) {
    const Problem& pr = pl.pr;
    const int N = pr.N;
    RH_HIP(rh::launch_resid_gate(b.rep, pr.explicit_error ? 1 : 0, b.gate, s));
    int64_t d[RHOSVD_MAX_ORDER];
    for (int n = 0; n < N; ++n) d[n] = pr.ranks[n];
    const void* src = out->core;
    void* bufs[2] = {b.ping, b.pong};
    for (int n = 0; n + 1 < N; ++n) {
        const int64_t L = prod(d, 0, n), T = prod(d, n + 1, N);
        void* dst = bufs[n % 2];
        RH_HIP(rh::launch_expand(pr.dbl, b.gate, src, out->factors[n], L,
                                 static_cast<int>(pr.dims[n]), pr.ranks[n], T, dst, s));
        d[n] = pr.dims[n];
        src = dst;
    }
    RH_HIP(rh::launch_resid(pr.dbl, b.gate, x, src, out->factors[N - 1], prod(pr.dims, 0, N - 1),
                            static_cast<int>(pr.dims[N - 1]), pr.ranks[N - 1], b.part_resid, b.rep,
                            s));
    return RHOSVD_OK;
}

int planning_cu(const rhosvd_ctx* ctx) { return ctx ? ctx->num_cu : 256; }

// The whole decomposition on a given workspace; `pl` is the caller's plan
// storage.  `too_small` is returned when the workspace cannot hold the plan.
int32_t decompose_on(rhosvd_ctx* ctx, const rhosvd_tensor* x, const rhosvd_params* p,
                            void* workspace, size_t ws_bytes, int32_t too_small,
                            const rhosvd_output* out, void* stream, Plan* pl) {
    if (!ctx || !out || !out->core || !out->factors || !workspace) return RHOSVD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return RHOSVD_EINVAL;
    Problem pr;
    int32_t rc = validate(x, p, &pr, true);
    if (rc != RHOSVD_OK) return rc;
    pr.kernels = ctx->kernels;
    for (int n = 0; n < pr.N; ++n)
        if (!out->factors[n]) return RHOSVD_EINVAL;
    // the grid is planned for a 256-CU part so that the workspace size does
    // not depend on the device the context was created on
    rc = build_plan(pr, planning_cu(nullptr), pl);
    if (rc != RHOSVD_OK) return rc;
    Buffers b;
    const size_t need = carve(*pl, nullptr, &b);
    if (ws_bytes < need) return too_small;
    carve(*pl, workspace, &b);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = -1;
    RH_HIP(hipGetDevice(&dev));
    if (dev != ctx->device) RH_HIP(hipSetDevice(ctx->device));
    rh::ReportInit ri{};
    ri.order = pr.N;
    for (int si = 0; si < pr.N; ++si) {
        const Step& st = pl->st[si];
        ri.k_used[st.n] = st.capped ? -st.K : st.K;
    }
    rc = RHOSVD_OK;
    hipError_t he = rh::launch_report_init(b.rep, ri, s);
    if (he != hipSuccess) rc = hip_fail(he);
    if (rc == RHOSVD_OK)
        rc = (pr.algo == RHOSVD_R_STHOSVD) ? run_r_sthosvd(*pl, b, x->data, out, s)
                                            : run_rp_hosvd(*pl, b, x->data, out, s);   // RP-HOSVD, RP-HOOI, R-PET
    if (rc == RHOSVD_OK) {
        he = rh::launch_sumsq(pr.dbl, out->core, pl->core_elems, b.part_ss, kSumsqBlocks, s);
        if (he == hipSuccess) he = rh::launch_reduce_ss(b.part_ss, kSumsqBlocks, &b.rep->norm_core2, s);
        if (he != hipSuccess) rc = hip_fail(he);
    }
    if (rc == RHOSVD_OK) rc = run_residual(*pl, b, x->data, out, s);
    if (rc == RHOSVD_OK && out->report) {
        he = rh::launch_copy_bytes(b.rep, out->report, sizeof(rhosvd_report), s);
        if (he != hipSuccess) rc = hip_fail(he);
    }
    if (dev != ctx->device) (void)hipSetDevice(dev);
    return rc;
}

// ---- fixed-precision R-STHOSVD (Section 5.1, the tolerance split of
// Algorithm 4) -----------------------------------------------------------

// The problem with every R_n = K_n = min(kmax, I_n, J_n): the largest tensors
// (and workspace) the adaptive path can meet.  ks receives the K_n.
int32_t adaptive_problem(const rhosvd_tensor* x, const rhosvd_adaptive_params* ap, int32_t* ks,
                         rhosvd_params* p) {
    if (!x || !ap || !x->dims) return RHOSVD_EINVAL;
    if (!(ap->eps > 0.0) || ap->kmax < 1 || ap->kmax > RHOSVD_MAX_SKETCH) return RHOSVD_EINVAL;
    if (x->order < 2 || x->order > RHOSVD_MAX_ORDER) return RHOSVD_EINVAL;
    const int N = x->order;
    int64_t d[RHOSVD_MAX_ORDER];
    for (int n = 0; n < N; ++n) {
        if (x->dims[n] < 1) return RHOSVD_EINVAL;
        d[n] = x->dims[n];
    }
    for (int n = 0; n < N; ++n) {
        const int64_t J = prod(d, 0, n) * prod(d, n + 1, N);
        const int64_t K = std::min<int64_t>(std::min<int64_t>(ap->kmax, d[n]), J);
        ks[n] = static_cast<int32_t>(K);
        d[n] = K;
    }
    *p = rhosvd_params{};
    p->algo = RHOSVD_R_STHOSVD;
    p->ranks = ks;
    p->oversample = 0;
    p->power_iters = ap->power_iters;
    p->seed = ap->seed;
    p->mode_order = nullptr;
    p->precision = ap->precision;
    p->flags = ap->flags;
    return RHOSVD_OK;
}

// The partials of pass g fit the buffers carved for the worst-case plan.
bool partials_fit(const Plan& pl, const Pass& g, bool gram) {
    const size_t y = static_cast<size_t>(g.grid) * g.K_pad * g.I_pad * pl.pr.elem;
    const size_t gg = gram ? static_cast<size_t>(g.grid) * g.K_pad * g.K_pad * pl.pr.elem : 0;
    return y <= pl.part_bytes && gg <= pl.part_bytes && g.grid <= pl.max_grid;
}

// Mode by mode: sketch, power steps, B and its Gram, all K eigenpairs and
// U = Q Ubar (K columns); the eigenvalues come to the host, which keeps the
// smallest R whose residual ||S||^2 - sum_{i <= R} sigma_i^2 is within the
// mode's share eps^2 ||X||^2 / N, and the truncation keeps R rows.
int32_t run_adaptive(rhosvd_ctx* ctx, Plan* pl, const Buffers& b, const rhosvd_tensor* x,
                     const rhosvd_adaptive_params* ap, const rhosvd_output* out,
                     int32_t* ranks_out, int32_t* met_out, hipStream_t s) {
    const Problem& pr = pl->pr;
    const bool dbl = pr.dbl;
    const int N = pr.N;
    const int cu = planning_cu(nullptr);
    int64_t d[RHOSVD_MAX_ORDER];
    for (int n = 0; n < N; ++n) d[n] = pr.dims[n];
    const void* src = x->data;
    double budget = 0.0;
    (void)ctx;
    for (int n = 0; n < N; ++n) {
        const int64_t I = d[n], T = prod(d, 0, N) / d[n];
        const int K = static_cast<int>(std::min<int64_t>(std::min<int64_t>(ap->kmax, I), T));
        const bool capped = K < ap->kmax;
        Pass gs, gp, gt, gtr;
        if (!plan_pass(rh::OP_SKETCH, dbl, pr.ct_sketch, 1, I, T, K, cu, &gs, pr.kernels) ||
            !plan_pass(rh::OP_POWER, dbl, pr.ct_power, 1, I, T, K, cu, &gp, pr.kernels) ||
            !plan_pass(rh::OP_TTM, dbl, pr.ct_ttm, 1, I, T, K, cu, &gt, pr.kernels))
            return RHOSVD_EUNSUPPORTED;
        if (!partials_fit(*pl, gs, false) || (pr.q > 0 && !partials_fit(*pl, gp, false)) ||
            !partials_fit(*pl, gt, true) || I * K > pl->maxIK || static_cast<int64_t>(K) * T > pl->maxB ||
            static_cast<int64_t>(K) * K > pl->maxKR || static_cast<int64_t>(K) * K > pl->maxKK ||
            static_cast<int64_t>(rh::evd_qwork_doubles(K, I)) > pl->maxQW)
            return RHOSVD_EUNSUPPORTED;
        double* nrm = n == 0 ? &b.rep->norm_x2 : b.part_resid;
        rh::KrArgs kr{};
        if (pr.kr) {
            // this mode's tables at the current extents (within the room the
            // worst case, every earlier R = K, reserved)
            for (int q = 0; q < N - 1; ++q) pl->kr_ext[n][q] = d[pl->kr_mode[n][q]];
            int modes[RHOSVD_MAX_ORDER], Ks[RHOSVD_MAX_ORDER];
            modes[n] = n;
            Ks[n] = K;
            const int32_t rf = fill_kr(*pl, b, n, n + 1, modes, Ks, s);
            if (rf != RHOSVD_OK) return rf;
            kr = kr_args(*pl, b, n, K, T);
        }
        int32_t rc = sketch_and_orthonormalize(*pl, b, src, gs, gp, n, 2u, nrm, b.qT, s, kr);
        if (rc != RHOSVD_OK) return rc;
        rc = ttm(*pl, gt, src, b.qT, b.B, b.part, s);
        if (rc != RHOSVD_OK) return rc;
        RH_HIP(rh::launch_gram_reduce(dbl, b.part, gt.grid, K, gt.K_pad, b.C, s));
        RH_HIP(rh::launch_evd_factor(dbl, b.C, K, &b.rep->flags, b.qT, I, K, 1, out->factors[n], b.M,
                                     &b.rep->sigma[n][0], b.u64, s));
        double sig[RHOSVD_MAX_K], nrm_h = 0.0;
        RH_HIP(hipStreamSynchronize(s));
        RH_HIP(hipMemcpy(sig, &b.rep->sigma[n][0], sizeof(double) * K, hipMemcpyDeviceToHost));
        RH_HIP(hipMemcpy(&nrm_h, nrm, sizeof(double), hipMemcpyDeviceToHost));
        if (n == 0) budget = ap->eps * ap->eps * nrm_h / N;
        int R = K;
        bool met = false;
        double kept = 0.0;
        for (int r = 1; r <= K; ++r) {
            kept += sig[r - 1] * sig[r - 1];
            if (nrm_h - kept <= budget) {
                R = r;
                met = true;
                break;
            }
        }
        ranks_out[n] = R;
        if (met_out) met_out[n] = met ? 1 : 0;
        RH_HIP(rh::launch_report_mode(b.rep, n, capped ? -K : K, R, s));
        if (!plan_pass(rh::OP_TTM, dbl, pr.ct_trunc, 1, K, T, R, cu, &gtr, pr.kernels))
            return RHOSVD_EUNSUPPORTED;
        void* dst = (n == N - 1) ? out->core : ((n % 2 == 0) ? b.ping : b.pong);
        if (n < N - 1 && R * T > ((n % 2 == 0) ? pl->ping : pl->pong)) return RHOSVD_EUNSUPPORTED;
        rh::TruncGeom tg;
        if (pr.kernels == RHOSVD_KERNELS_AUTO && rh::plan_trunc(dbl, K, T, R, cu, false, &tg)) {
            RH_HIP(rh::launch_trunc(dbl, tg, b.B, b.M, dst, s));
        } else {
            rc = ttm(*pl, gtr, b.B, b.M, dst, nullptr, s, 1);
            if (rc != RHOSVD_OK) return rc;
        }
        src = dst;
        d[n] = R;
    }
    // the chosen ranks are the problem's ranks from here on (core norm,
    // residual)
    pl->core_elems = prod(d, 0, N);
    for (int n = 0; n < N; ++n) pl->pr.ranks[n] = ranks_out[n];
    return RHOSVD_OK;
}

int32_t decompose_adaptive_on(rhosvd_ctx* ctx, const rhosvd_tensor* x,
                              const rhosvd_adaptive_params* ap, void* workspace, size_t ws_bytes,
                              const rhosvd_output* out, int32_t* ranks_out, int32_t* met_out,
                              void* stream, Plan* pl) {
    if (!ctx || !out || !out->core || !out->factors || !workspace || !ranks_out) return RHOSVD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return RHOSVD_EINVAL;
    int32_t ks[RHOSVD_MAX_ORDER];
    rhosvd_params p;
    int32_t rc = adaptive_problem(x, ap, ks, &p);
    if (rc != RHOSVD_OK) return rc;
    Problem pr;
    rc = validate(x, &p, &pr, true);
    if (rc != RHOSVD_OK) return rc;
    pr.kernels = ctx->kernels;
    for (int n = 0; n < pr.N; ++n)
        if (!out->factors[n]) return RHOSVD_EINVAL;
    rc = build_plan(pr, planning_cu(nullptr), pl);
    if (rc != RHOSVD_OK) return rc;
    Buffers b;
    const size_t need = carve(*pl, nullptr, &b);
    if (ws_bytes < need) return RHOSVD_ENOMEM;
    carve(*pl, workspace, &b);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = -1;
    RH_HIP(hipGetDevice(&dev));
    if (dev != ctx->device) RH_HIP(hipSetDevice(ctx->device));
    rh::ReportInit ri{};
    ri.order = pr.N;
    for (int n = 0; n < pr.N; ++n) ri.k_used[n] = ks[n];
    rc = RHOSVD_OK;
    hipError_t he = rh::launch_report_init(b.rep, ri, s);
    if (he != hipSuccess) rc = hip_fail(he);
    if (rc == RHOSVD_OK) rc = run_adaptive(ctx, pl, b, x, ap, out, ranks_out, met_out, s);
    if (rc == RHOSVD_OK) {
        he = rh::launch_sumsq(pr.dbl, out->core, pl->core_elems, b.part_ss, kSumsqBlocks, s);
        if (he == hipSuccess) he = rh::launch_reduce_ss(b.part_ss, kSumsqBlocks, &b.rep->norm_core2, s);
        if (he != hipSuccess) rc = hip_fail(he);
    }
    if (rc == RHOSVD_OK) rc = run_residual(*pl, b, x->data, out, s);
    if (rc == RHOSVD_OK && out->report) {
        he = rh::launch_copy_bytes(b.rep, out->report, sizeof(rhosvd_report), s);
        if (he != hipSuccess) rc = hip_fail(he);
    }
    if (rc == RHOSVD_OK) {
        he = hipStreamSynchronize(s);
        if (he != hipSuccess) rc = hip_fail(he);
    }
    if (dev != ctx->device) (void)hipSetDevice(dev);
    return rc;
}

}  // namespace

namespace rh {

// rhosvd_decompose on a caller-given fixed workspace, with the plan on the
// stack (no allocation of any kind); `too_small` is returned when the plan
// does not fit.
int32_t decompose_fixed(rhosvd_ctx* ctx, const rhosvd_tensor* x,
                                        const rhosvd_params* p, void* ws, size_t ws_bytes,
                                        int32_t too_small, const rhosvd_output* out,
                                        void* stream) {
    Plan pl;
    return decompose_on(ctx, x, p, ws, ws_bytes, too_small, out, stream, &pl);
}

void* ctx_scratch(const rhosvd_ctx* ctx) { return ctx ? ctx->scratch : nullptr; }

}  // namespace rh

extern "C" {

const char* rhosvd_status_string(int32_t status) {
    switch (status) {
        case RHOSVD_OK: return "ok";
        case RHOSVD_EINVAL: return "invalid argument";
        case RHOSVD_ENOMEM: return "workspace too small";
        case RHOSVD_EHIP: return "HIP runtime error";
        case RHOSVD_ENUMERIC: return "numerical failure";
        case RHOSVD_EBUSY: return "busy";
        case RHOSVD_EUNSUPPORTED: return "unsupported problem size";
        case RHOSVD_ESCRATCH: return "problem exceeds the fixed no-alloc scratch";
        default: return "unknown status";
    }
}

int32_t rhosvd_last_hip_error(void) { return g_last_hip; }

int32_t rhosvd_create(rhosvd_ctx** ctx, int32_t device) {
    if (!ctx) return RHOSVD_EINVAL;
    *ctx = nullptr;
    int count = 0;
    RH_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return RHOSVD_EINVAL;
    hipDeviceProp_t prop;
    RH_HIP(hipGetDeviceProperties(&prop, device));
    void* sp = nullptr;
    const int32_t rs = rh::noalloc_scratch_address(device, &sp);
    if (rs != RHOSVD_OK) return rs;
    rhosvd_ctx* c = new (std::nothrow) rhosvd_ctx;
    if (!c) return RHOSVD_ENOMEM;
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    c->lds_per_block = prop.sharedMemPerBlock;
    c->kernels = RHOSVD_KERNELS_AUTO;
    c->scratch = sp;
    *ctx = c;
    return RHOSVD_OK;
}

void rhosvd_destroy(rhosvd_ctx* ctx) { delete ctx; }

int32_t rhosvd_set_option(rhosvd_ctx* ctx, int32_t option, int64_t value) {
    if (!ctx) return RHOSVD_EINVAL;
    if (option == RHOSVD_OPTION_KERNELS) {
        if (value != RHOSVD_KERNELS_AUTO && value != RHOSVD_KERNELS_TILED) return RHOSVD_EINVAL;
        ctx->kernels = static_cast<int>(value);
        return RHOSVD_OK;
    }
    return RHOSVD_EINVAL;
}


int32_t rhosvd_workspace_size(const rhosvd_tensor* x, const rhosvd_params* p, size_t* bytes) {
    if (!bytes) return RHOSVD_EINVAL;
    Problem pr;
    int32_t rc = validate(x, p, &pr, false);
    if (rc != RHOSVD_OK) return rc;
    Plan* pl = new (std::nothrow) Plan;
    if (!pl) return RHOSVD_ENOMEM;
    rc = build_plan(pr, planning_cu(nullptr), pl);
    if (rc == RHOSVD_OK) {
        Buffers b;
        *bytes = carve(*pl, nullptr, &b);
    }
    delete pl;
    return rc;
}

int32_t rhosvd_decompose(rhosvd_ctx* ctx, const rhosvd_tensor* x, const rhosvd_params* p,
                         void* workspace, size_t ws_bytes, const rhosvd_output* out,
                         void* stream) {
    Plan* pl = new (std::nothrow) Plan;
    if (!pl) return RHOSVD_ENOMEM;
    const int32_t rc = decompose_on(ctx, x, p, workspace, ws_bytes, RHOSVD_ENOMEM, out, stream, pl);
    delete pl;
    return rc;
}

int32_t rhosvd_adaptive_workspace_size(const rhosvd_tensor* x, const rhosvd_adaptive_params* p,
                                       size_t* bytes) {
    if (!bytes) return RHOSVD_EINVAL;
    int32_t ks[RHOSVD_MAX_ORDER];
    rhosvd_params fp;
    const int32_t rc = adaptive_problem(x, p, ks, &fp);
    if (rc != RHOSVD_OK) return rc;
    return rhosvd_workspace_size(x, &fp, bytes);
}

int32_t rhosvd_decompose_adaptive(rhosvd_ctx* ctx, const rhosvd_tensor* x,
                                  const rhosvd_adaptive_params* p, void* workspace,
                                  size_t ws_bytes, const rhosvd_output* out, int32_t* ranks_out,
                                  int32_t* met_out, void* stream) {
    Plan* pl = new (std::nothrow) Plan;
    if (!pl) return RHOSVD_ENOMEM;
    const int32_t rc = decompose_adaptive_on(ctx, x, p, workspace, ws_bytes, out, ranks_out,
                                             met_out, stream, pl);
    delete pl;
    return rc;
}

double rhosvd_report_rel_error(const rhosvd_report* r) {
    if (!r || !(r->norm_x2 > 0.0)) return NAN;
    if (r->flags & RHOSVD_FLAG_E_EXPLICIT) return std::sqrt(r->resid2 / r->norm_x2);
    const double d = r->norm_x2 - r->norm_core2;
    return std::sqrt((d > 0.0 ? d : 0.0) / r->norm_x2);
}

// ---- step-level entry points ----------------------------------------------

size_t rhosvd_step_workspace_size(int64_t I, int32_t K, int64_t J) {
    (void)J;
    if (I < 1 || K < 1) return 0;
    const size_t Ip = static_cast<size_t>((I + 15) / 16 * 16), Kp = static_cast<size_t>((K + 15) / 16 * 16);
    const size_t G = 512;
    const size_t big = Ip > Kp ? Ip : Kp;
    return 256 + G * Kp * big * sizeof(double) + 256 + G * sizeof(double) + 256 +
           kSumsqBlocks * sizeof(double) + 256;
}

static int32_t step_ws(void* ws, size_t bytes, int64_t I, int32_t K, void** part, double** ss) {
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0) return RHOSVD_EINVAL;
    if (bytes < rhosvd_step_workspace_size(I, K, 0)) return RHOSVD_ENOMEM;
    Carver cv(ws);
    const size_t Ip = static_cast<size_t>((I + 15) / 16 * 16), Kp = static_cast<size_t>((K + 15) / 16 * 16);
    const size_t big = Ip > Kp ? Ip : Kp;
    *part = cv.take<void>(512 * Kp * big * sizeof(double));
    const size_t nss = 512 > kSumsqBlocks ? 512 : kSumsqBlocks;
    *ss = cv.take<double>(nss * sizeof(double));
    return RHOSVD_OK;
}

int32_t rhosvd_omega_fill(rhosvd_ctx* ctx, uint64_t seed, int32_t mode, int32_t tag, int64_t J,
                          int32_t K, int32_t dtype, void* out, void* stream) {
    if (!ctx || !out || J < 1 || K < 1 || (dtype != RHOSVD_F32 && dtype != RHOSVD_F64))
        return RHOSVD_EINVAL;
    RH_HIP(rh::launch_omega_fill(dtype == RHOSVD_F64, seed, mode, tag, J, K, out,
                                 static_cast<hipStream_t>(stream)));
    return RHOSVD_OK;
}

static void step_cts(int32_t precision, int* s, int* p, int* t) {
    if (precision == RHOSVD_PREC_BF16 || precision == RHOSVD_PREC_FP8E4M3) {
        *s = precision == RHOSVD_PREC_BF16 ? rh::CT_BF16 : rh::CT_FP8;
        *p = rh::CT_BF16X3;
        *t = rh::CT_BF16X3;
    } else {
        *s = *p = *t = rh::CT_F32;
    }
}

static int32_t check_view(int32_t dtype, int32_t precision, int64_t L, int64_t I, int64_t T,
                          int32_t K) {
    if (dtype != RHOSVD_F32 && dtype != RHOSVD_F64) return RHOSVD_EINVAL;
    if (L < 1 || I < 1 || T < 1 || K < 1 || K > RHOSVD_MAX_K) return RHOSVD_EINVAL;
    if (dtype == RHOSVD_F64 && precision != RHOSVD_PREC_F64) return RHOSVD_EINVAL;
    if (dtype == RHOSVD_F32 && precision != RHOSVD_PREC_F32 && precision != RHOSVD_PREC_BF16 &&
        precision != RHOSVD_PREC_FP8E4M3)
        return RHOSVD_EINVAL;
    return RHOSVD_OK;
}

static int32_t sketch_step(rhosvd_ctx* ctx, const void* src, int32_t dtype, int32_t precision,
                           int64_t L, int64_t I, int64_t T, int32_t K, uint64_t seed, int32_t mode,
                           int32_t tag, const rh::KrArgs& kr, double* y, double* norm2,
                           void* workspace, size_t ws_bytes, void* stream);

int32_t rhosvd_sketch(rhosvd_ctx* ctx, const void* src, int32_t dtype, int32_t precision,
                      int64_t L, int64_t I, int64_t T, int32_t K, uint64_t seed, int32_t mode,
                      int32_t tag, double* y, double* norm2, void* workspace, size_t ws_bytes,
                      void* stream) {
    return sketch_step(ctx, src, dtype, precision, L, I, T, K, seed, mode, tag, rh::KrArgs{}, y,
                       norm2, workspace, ws_bytes, stream);
}

int32_t rhosvd_sketch_kr(rhosvd_ctx* ctx, const void* src, int32_t dtype, int32_t precision,
                         int64_t L, int64_t I, int64_t T, int32_t K, const void* const* tabs,
                         const int64_t* ext, int32_t nq, double* y, double* norm2,
                         void* workspace, size_t ws_bytes, void* stream) {
    if (!tabs || !ext || nq < 1 || nq > RHOSVD_MAX_ORDER - 1 || K < 1) return RHOSVD_EINVAL;
    rh::KrArgs kr{};
    kr.nq = nq;
    kr.K = K;
    kr.J = L * T;
    int64_t prodx = 1;
    for (int q = 0; q < nq; ++q) {
        if (!tabs[q] || ext[q] < 1 || ext[q] > (int64_t(1) << 31) - 1) return RHOSVD_EINVAL;
        kr.tab[q] = tabs[q];
        kr.ext[q] = static_cast<int>(ext[q]);
        prodx *= ext[q];
        if (prodx > (int64_t(1) << 32)) return RHOSVD_EINVAL;
    }
    if (prodx != L * T) return RHOSVD_EINVAL;
    return sketch_step(ctx, src, dtype, precision, L, I, T, K, 0, 0, 0, kr, y, norm2, workspace,
                       ws_bytes, stream);
}

static int32_t sketch_step(rhosvd_ctx* ctx, const void* src, int32_t dtype, int32_t precision,
                           int64_t L, int64_t I, int64_t T, int32_t K, uint64_t seed, int32_t mode,
                           int32_t tag, const rh::KrArgs& kr, double* y, double* norm2,
                           void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx || !src || !y) return RHOSVD_EINVAL;
    int32_t rc = check_view(dtype, precision, L, I, T, K);
    if (rc != RHOSVD_OK) return rc;
    Pass g;
    const bool dbl = dtype == RHOSVD_F64;
    int ct_s, ct_p, ct_t;
    step_cts(precision, &ct_s, &ct_p, &ct_t);
    if (!plan_pass(rh::OP_SKETCH, dbl, ct_s, L, I, T, K, 256, &g, ctx->kernels)) return RHOSVD_EUNSUPPORTED;
    void* part;
    double* ss;
    rc = step_ws(workspace, ws_bytes, I, K, &part, &ss);
    if (rc != RHOSVD_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rh::StreamArgs a{};
    a.src = src;
    a.part_y = part;
    a.part_ss = norm2 ? ss : nullptr;
    a.seed = seed;
    a.mode = static_cast<uint32_t>(mode);
    a.tag = static_cast<uint32_t>(tag);
    a.kr = kr;
    RH_HIP(launch_pass(g, a, s));
    RH_HIP(rh::launch_reduce_y(dbl, part, g.grid, static_cast<int>(I), K, g.I_pad, g.K_pad, y, s));
    if (norm2) RH_HIP(rh::launch_reduce_ss(ss, g.grid, norm2, s));
    return RHOSVD_OK;
}

static int32_t plan_sketch_all(int32_t order, const int64_t* dims, const int32_t* K, int32_t dtype,
                               rh::AllModeArgs* a) {
    if (order < 2 || order > RHOSVD_MAX_ORDER || !dims || !K) return RHOSVD_EINVAL;
    if (dtype != RHOSVD_F32 && dtype != RHOSVD_F64) return RHOSVD_EINVAL;
    int Ks[RHOSVD_MAX_ORDER];
    double total = 1.0;
    for (int n = 0; n < order; ++n) {
        if (dims[n] < 1 || K[n] < 1) return RHOSVD_EINVAL;
        total *= static_cast<double>(dims[n]);
        Ks[n] = K[n];
    }
    if (total > 4.0e18) return RHOSVD_EINVAL;
    for (int n = 0; n < order; ++n)
        if (K[n] > RHOSVD_MAX_SKETCH || K[n] > total / dims[n]) return RHOSVD_EUNSUPPORTED;
    if (!rh::plan_allmode(order, dims, Ks, 256, dtype == RHOSVD_F64 ? 8 : 4, a))
        return RHOSVD_EUNSUPPORTED;
    return RHOSVD_OK;
}

size_t rhosvd_sketch_all_workspace_size(int32_t order, const int64_t* dims, const int32_t* K,
                                        int32_t dtype) {
    rh::AllModeArgs a;
    if (plan_sketch_all(order, dims, K, dtype, &a) != RHOSVD_OK) return 0;
    const size_t elem = dtype == RHOSVD_F64 ? 8 : 4;
    return 256 + static_cast<size_t>(a.grid) * a.S * elem + 256 + a.grid * sizeof(double) + 256;
}

int32_t rhosvd_sketch_all(rhosvd_ctx* ctx, const void* src, int32_t dtype, int32_t order,
                          const int64_t* dims, const int32_t* K, uint64_t seed, int32_t tag,
                          double* y, double* norm2, void* workspace, size_t ws_bytes,
                          void* stream) {
    if (!ctx || !src || !y || !workspace) return RHOSVD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return RHOSVD_EINVAL;
    rh::AllModeArgs a;
    const int32_t rc = plan_sketch_all(order, dims, K, dtype, &a);
    if (rc != RHOSVD_OK) return rc;
    if (ws_bytes < rhosvd_sketch_all_workspace_size(order, dims, K, dtype)) return RHOSVD_ENOMEM;
    const bool dbl = dtype == RHOSVD_F64;
    Carver cv(workspace);
    a.part = cv.take<void>(static_cast<size_t>(a.grid) * a.S * (dbl ? 8 : 4));
    a.part_ss = cv.take<double>(a.grid * sizeof(double));
    a.x = src;
    a.seed = seed;
    a.tag = static_cast<uint32_t>(tag);
    hipStream_t s = static_cast<hipStream_t>(stream);
    RH_HIP(rh::launch_allmode(dbl, a, s));
    RH_HIP(rh::launch_allmode_reduce(dbl, a, y, s));
    if (norm2) RH_HIP(rh::launch_reduce_ss(a.part_ss, a.grid, norm2, s));
    return RHOSVD_OK;
}

int32_t rhosvd_power(rhosvd_ctx* ctx, const void* src, int32_t dtype, int32_t precision,
                     int64_t L, int64_t I, int64_t T, int32_t K, const void* q_in, double* y,
                     void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx || !src || !q_in || !y) return RHOSVD_EINVAL;
    int32_t rc = check_view(dtype, precision, L, I, T, K);
    if (rc != RHOSVD_OK) return rc;
    Pass g;
    const bool dbl = dtype == RHOSVD_F64;
    int ct_s, ct_p, ct_t;
    step_cts(precision, &ct_s, &ct_p, &ct_t);
    if (!plan_pass(rh::OP_POWER, dbl, ct_p, L, I, T, K, 256, &g, ctx->kernels)) return RHOSVD_EUNSUPPORTED;
    void* part;
    double* ss;
    rc = step_ws(workspace, ws_bytes, I, K, &part, &ss);
    if (rc != RHOSVD_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rh::StreamArgs a{};
    a.src = src;
    a.mat = q_in;
    a.part_y = part;
    RH_HIP(launch_pass(g, a, s));
    RH_HIP(rh::launch_reduce_y(dbl, part, g.grid, static_cast<int>(I), K, g.I_pad, g.K_pad, y, s));
    return RHOSVD_OK;
}

int32_t rhosvd_ttm(rhosvd_ctx* ctx, const void* src, int32_t dtype, int32_t precision, int64_t L,
                   int64_t I, int64_t T, int32_t Kout, const void* m, void* out, double* gram,
                   double* norm2, void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx || !src || !out) return RHOSVD_EINVAL;
    int32_t rc = check_view(dtype, precision, L, I, T, Kout);
    if (rc != RHOSVD_OK) return rc;
    if (!m && Kout != I) return RHOSVD_EINVAL;
    Pass g;
    const bool dbl = dtype == RHOSVD_F64;
    int ct_s, ct_p, ct_t;
    step_cts(precision, &ct_s, &ct_p, &ct_t);
    if (!plan_pass(rh::OP_TTM, dbl, ct_t, L, I, T, Kout, 256, &g, ctx->kernels)) return RHOSVD_EUNSUPPORTED;
    void* part;
    double* ss;
    rc = step_ws(workspace, ws_bytes, I, Kout, &part, &ss);
    if (rc != RHOSVD_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rh::StreamArgs a{};
    a.src = src;
    a.mat = m;
    a.out = out;
    a.part_g = gram ? part : nullptr;
    RH_HIP(launch_pass(g, a, s));
    if (gram) RH_HIP(rh::launch_gram_reduce(dbl, part, g.grid, Kout, g.K_pad, gram, s));
    if (norm2) {
        RH_HIP(rh::launch_sumsq(dbl, out, L * static_cast<int64_t>(Kout) * T, ss, kSumsqBlocks, s));
        RH_HIP(rh::launch_reduce_ss(ss, kSumsqBlocks, norm2, s));
    }
    return RHOSVD_OK;
}

int32_t rhosvd_truncate_rotated(rhosvd_ctx* ctx, int32_t dtype, const void* b, int32_t K, int64_t J,
                                const void* m, int32_t R, void* out, void* stream) {
    if (!ctx || !b || !m || !out) return RHOSVD_EINVAL;
    if (dtype != RHOSVD_F32 && dtype != RHOSVD_F64) return RHOSVD_EINVAL;
    if (K < 1 || R < 1 || R > K || J < 1) return RHOSVD_EINVAL;
    rh::TruncGeom tg;
    if (!rh::plan_trunc(dtype == RHOSVD_F64, K, J, R, ctx->num_cu, true, &tg)) return RHOSVD_EUNSUPPORTED;
    RH_HIP(rh::launch_trunc(dtype == RHOSVD_F64, tg, b, m, out, static_cast<hipStream_t>(stream)));
    return RHOSVD_OK;
}

int32_t rhosvd_orthonormalize(rhosvd_ctx* ctx, const double* y, int64_t I, int32_t K,
                              int32_t dtype, void* q_out, double* work, uint32_t* flags,
                              void* stream) {
    if (!ctx || !y || !q_out || !work) return RHOSVD_EINVAL;
    if (dtype != RHOSVD_F32 && dtype != RHOSVD_F64) return RHOSVD_EINVAL;
    if (K < 1 || I < K || I > (int64_t)1 << 30) return RHOSVD_EINVAL;
    if (K > kMaxSmallK) return RHOSVD_EUNSUPPORTED;
    RH_HIP(rh::launch_cqr(y, I, K, dtype == RHOSVD_F64, q_out, work, flags,
                          static_cast<hipStream_t>(stream)));
    return RHOSVD_OK;
}

int32_t rhosvd_sym_evd(rhosvd_ctx* ctx, const double* c, int32_t K, double* v, double* lambda,
                       uint32_t* flags, void* stream) {
    if (!ctx || !c || !v || !lambda || K < 1) return RHOSVD_EINVAL;
    if (K > kMaxSmallK) return RHOSVD_EUNSUPPORTED;
    RH_HIP(rh::launch_evd(c, K, v, lambda, flags, static_cast<hipStream_t>(stream)));
    return RHOSVD_OK;
}

}  // extern "C"

// ---- batched decomposition ------------------------------------------------
// Many small tensors, one launch per step for the whole batch: every
// streaming pass, reduction, QR and EVD of mode step s of every item goes
// into one launch driven by a device table of jobs (grouped by the template
// the small kernels need), and the whole sequence is captured once into a
// HIP graph and replayed.  Each item keeps the buffers of its own
// single-tensor plan (carved from its own region of the workspace) and runs
// the workgroup-tiled streaming kernels, so an item's arithmetic depends only
// on its own shape and the tuned tile parameters, never on the other items.

namespace {

constexpr int kBatchUnits = 64;          // most workgroups per item per pass
// on the wave kernels: measured on the 512-tensor workload, 16 workgroups per
// item (each wave then takes ~4x the blocks, its pipeline's start and the
// partial sums amortised over them) ran 23.6 ms (bf16) / 26.0 ms (FP32)
// against 26.8 / 30.6 with 64 and 29.1 (FP32) with 8
constexpr int kBatchWaveUnits = 16;
// on the column and truncation kernels, with each launch's jobs in decreasing
// size (the largest items start first, the small ones fill the tail): at most
// 12 workgroups per item and at least 16 column blocks per workgroup, 11.3 ms
// on the 512-tensor workload (bf16) against 12.6 with 16 and 4, 13.3 with the
// jobs in item order
constexpr int kBatchColUnits = 12;
constexpr int kBatchColMinBlocks = 16;
// most parallel branches of one group in the captured graph: the largest
// launches get one each, the smallest follow one another on the caller's
// stream (with up to ten branches the graph's tenth launch waited for all
// the others)
constexpr size_t kBatchBranches = 8;

enum BatchKind { BK_STREAM, BK_REDUCE, BK_QR, BK_EVD, BK_INIT, BK_NORMX, BK_FINISH, BK_WAVE, BK_COL, BK_TRUNC };

struct BatchLaunch {
    int kind = 0, op = 0, njobs = 0, sel = 0;
    int grp = 0;                      // launches of one pass, QR or EVD step (disjoint
                                      // items, so independent of each other) share a
                                      // nonzero group
    double work = 0.0;                // size estimate that orders a group's launches
    int ct = 0, var = 0;              // BK_WAVE: compute type and shape of the instantiation;
                                      // BK_COL: flag (Gram / sum of squares) and shape;
                                      // BK_TRUNC: row tiles and step bound
    size_t lds = 0, off = 0;
};

// Per pass of an item: the wave kernel when an FP32 item's shape has a
// batched instantiation (one 16-column block per wave, up to kBatchWaveUnits
// workgroups), else the tiled geometry with the tuned tile width cap and
// tiles per workgroup.  Either depends on the item's own shape only.
void batch_pass(Pass* p, int op, bool dbl, int ct, int elem, int64_t I, int64_t T, int K, int cmax,
                int tpu) {
    p->op = op;
    p->dbl = dbl;
    p->I = I;
    p->K = K;
    if (op == rh::OP_SKETCH && ct == rh::CT_FP8) ct = rh::CT_BF16;
    // bf16-path passes of modes up to 256 rows on the column kernels (32
    // columns per wave), as a single decomposition runs them
    rh::ColGeom cg;
    if (!dbl && rh::plan_col_batch(op, ct, I, T, K, &cg)) {
        int64_t units = (cg.nblocks + kBatchColMinBlocks - 1) / kBatchColMinBlocks;
        if (units > kBatchColUnits) units = kBatchColUnits;
        if (units < 1) units = 1;
        cg.grid = static_cast<int>(units);
        p->cg = cg;
        p->kind = PASS_COL;
        p->grid = cg.grid;
        p->I_pad = cg.I_pad;
        p->K_pad = cg.K_pad;
        return;
    }
    rh::WGeom wg;
    if (!dbl && rh::wave_batch_ct(op, ct) && rh::plan_wave(op, ct, 1, I, T, K, 256, &wg) &&
        rh::wave_batch_variant(wg) >= 0) {
        int64_t units = (wg.nblocks + 3) / 4;
        if (units > kBatchWaveUnits) units = kBatchWaveUnits;
        if (units < 1) units = 1;
        wg.grid = static_cast<int>(units);
        p->wg = wg;
        p->kind = PASS_WAVE;
        p->grid = wg.grid;
        p->I_pad = wg.IB * 16;
        p->K_pad = wg.NB * 16;
        return;
    }
    rh::StreamGeom g;
    if (!rh::plan_stream(op, elem, 1, I, T, K, 256, &g, cmax)) return;
    int64_t units = (g.ntiles + tpu - 1) / tpu;
    if (units > kBatchUnits) units = kBatchUnits;
    if (units < 1) units = 1;
    g.grid = static_cast<int>(units);
    p->sg = g;
    p->kind = PASS_TILED;
    p->grid = g.grid;
    p->I_pad = g.I_pad;
    p->K_pad = g.K_pad;
}

void batch_geometry(Plan* pl, int cmax, int tpu) {
    const Problem& pr = pl->pr;
    const int elem = static_cast<int>(pr.elem);
    for (int s = 0; s < pr.N; ++s) {
        Step& st = pl->st[s];
        batch_pass(&st.gs, rh::OP_SKETCH, pr.dbl, pr.ct_sketch, elem, st.I, st.T, st.K, cmax, tpu);
        batch_pass(&st.gp, rh::OP_POWER, pr.dbl, pr.ct_power, elem, st.I, st.T, st.K, cmax, tpu);
        batch_pass(&st.gt, rh::OP_TTM, pr.dbl, pr.ct_ttm, elem, st.I, st.T, st.K, cmax, tpu);
        // the truncation (rotated: the batch requires it) on its own kernel
        rh::TruncGeom tg;
        if (rh::plan_trunc(pr.dbl, st.K, st.T, st.R, 256, true, &tg)) {
            Pass* p = &st.gtr;
            p->op = rh::OP_TTM;
            p->dbl = pr.dbl;
            p->I = st.K;
            p->K = st.R;
            int64_t units = ((st.T + 63) / 64 + 3) / 4;
            if (units > kBatchColUnits) units = kBatchColUnits;
            if (units < 1) units = 1;
            tg.grid = static_cast<int>(units);
            p->tg = tg;
            p->kind = PASS_TRUNC;
            p->grid = tg.grid;
            p->I_pad = p->K_pad = 0;
        } else {
            batch_pass(&st.gtr, rh::OP_TTM, pr.dbl, pr.ct_trunc, elem, st.K, st.T, st.R, cmax, tpu);
        }
    }
}

}  // namespace

struct rhosvd_batch {
    rhosvd_ctx* ctx = nullptr;
    int n = 0, N = 0, maxq = 0;
    bool dbl = false;
    std::vector<Plan*> plans;
    std::vector<size_t> region;              // offset of each item's region
    std::vector<const void*> x;
    std::vector<void*> core, report;
    std::vector<std::vector<void*>> factors;
    size_t tables_cap = 0, ws_bytes = 0;
    unsigned char* ws = nullptr;
    std::vector<BatchLaunch> prog;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // side streams (default priority) and events that fork the launches of one
    // group into parallel branches of the captured graph
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> joins;
    hipEvent_t fork = nullptr;
    ~rhosvd_batch() {
        for (Plan* p : plans) delete p;
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipStream_t t : side) (void)hipStreamDestroy(t);
        for (hipEvent_t e : joins) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
    }
};

namespace {

// Host image of the device tables, appended launch by launch.
struct TableWriter {
    std::vector<unsigned char> bytes;
    template <typename J>
    size_t put(const std::vector<J>& jobs) {
        size_t off = (bytes.size() + 255) & ~static_cast<size_t>(255);
        bytes.resize(off + jobs.size() * sizeof(J));
        std::memcpy(bytes.data() + off, jobs.data(), jobs.size() * sizeof(J));
        return off;
    }
};

// The launch program of the whole batch (and its tables) for the bound
// workspace, with the current tile parameters of every plan.
void build_program(rhosvd_batch* B, TableWriter* tw) {
    B->prog.clear();
    const int n = B->n, N = B->N;
    std::vector<Buffers> bufs(n);
    for (int i = 0; i < n; ++i) carve(*B->plans[i], B->ws + B->region[i], &bufs[i]);
    std::vector<const void*> cur(B->x.begin(), B->x.end());
    int cur_grp = 0;
    // a group's launches (the tail of the program from `start`) by decreasing size
    auto order_group = [&](size_t start) {
        std::stable_sort(B->prog.begin() + static_cast<std::ptrdiff_t>(start), B->prog.end(),
                         [](const BatchLaunch& a, const BatchLaunch& b) { return a.work > b.work; });
    };
    auto add_stream = [&](int op, std::vector<rh::StreamJob>& jobs) {
        if (jobs.empty()) return;
        BatchLaunch L;
        L.kind = BK_STREAM;
        L.op = op;
        L.grp = cur_grp;
        L.work = static_cast<double>(jobs.size());
        L.njobs = static_cast<int>(jobs.size());
        for (auto& j : jobs) {
            L.sel = std::max(L.sel, j.units);
            L.lds = std::max(L.lds, j.g.lds_bytes);
        }
        L.off = tw->put(jobs);
        B->prog.push_back(L);
    };
    // one pass of every item: the tiled ones in one launch, the wave ones in
    // one launch per (compute type, shape) of the batched instantiations
    struct PassJob {
        const Pass* p;
        rh::StreamArgs a;
    };
    auto add_pass = [&](int op, const std::vector<PassJob>& jobs) {
        ++cur_grp;
        const size_t start = B->prog.size();
        std::vector<rh::StreamJob> tiled;
        std::map<std::pair<int, int>, std::vector<rh::WaveJob>> wave;
        std::map<std::pair<int, int>, std::vector<rh::ColJob>> col;
        std::map<std::pair<int, int>, std::vector<rh::TruncJob>> trunc;
        for (const PassJob& pj : jobs) {
            if (pj.p->kind == PASS_TRUNC) {
                rh::TruncJob t{};
                t.b = pj.a.src;
                t.m = pj.a.mat;
                t.out = pj.a.out;
                t.K = pj.p->tg.K;
                t.R = pj.p->tg.R;
                t.J = pj.p->tg.J;
                t.units = pj.p->grid;
                trunc[{pj.p->tg.rb, rh::trunc_kqm(t.K)}].push_back(t);
            } else if (pj.p->kind == PASS_COL) {
                rh::ColJob c{};
                c.g = pj.p->cg;
                c.a = pj.a;
                c.units = pj.p->grid;
                const int flag = (op == rh::OP_SKETCH) ? (pj.a.part_ss != nullptr)
                                                       : (op == rh::OP_TTM && pj.a.part_g != nullptr);
                col[{flag, pj.p->cg.variant}].push_back(c);
            } else if (pj.p->kind == PASS_WAVE) {
                rh::WaveJob w{};
                w.g = pj.p->wg;
                w.a = pj.a;
                w.units = pj.p->grid;
                w.want_ss = pj.a.part_ss != nullptr;
                w.want_gram = pj.a.part_g != nullptr;
                wave[{pj.p->wg.ct, rh::wave_batch_variant(pj.p->wg)}].push_back(w);
            } else {
                rh::StreamJob j{};
                j.g = pj.p->sg;
                j.units = pj.p->grid;
                j.a = pj.a;
                tiled.push_back(j);
            }
        }
        add_stream(op, tiled);
        for (auto& kv : trunc) {
            std::stable_sort(kv.second.begin(), kv.second.end(), [](const rh::TruncJob& a, const rh::TruncJob& b) {
                return a.J > b.J;
            });
            BatchLaunch L;
            L.kind = BK_TRUNC;
            L.op = op;
            L.grp = cur_grp;
            L.ct = kv.first.first;
            L.var = kv.first.second;
            L.njobs = static_cast<int>(kv.second.size());
            for (auto& t : kv.second) {
                L.work += static_cast<double>(t.K) * static_cast<double>(t.J);
                L.sel = std::max(L.sel, t.units);
                const size_t lds = rh::trunc_lds_bytes(t.K, B->dbl);
                L.lds = std::max(L.lds, lds);
            }
            L.off = tw->put(kv.second);
            B->prog.push_back(L);
        }
        for (auto& kv : col) {
            std::stable_sort(kv.second.begin(), kv.second.end(), [](const rh::ColJob& a, const rh::ColJob& b) {
                return a.g.I * a.g.J > b.g.I * b.g.J;
            });
            BatchLaunch L;
            L.kind = BK_COL;
            L.op = op;
            L.grp = cur_grp;
            L.ct = kv.first.first;
            L.var = kv.first.second;
            L.njobs = static_cast<int>(kv.second.size());
            for (auto& c : kv.second) {
                L.work += static_cast<double>(c.g.I) * static_cast<double>(c.g.J);
                L.sel = std::max(L.sel, c.units);
                L.lds = std::max(L.lds, c.g.lds_bytes);
            }
            L.off = tw->put(kv.second);
            B->prog.push_back(L);
        }
        for (auto& kv : wave) {
            std::stable_sort(kv.second.begin(), kv.second.end(), [](const rh::WaveJob& a, const rh::WaveJob& b) {
                return a.g.I * a.g.J > b.g.I * b.g.J;
            });
            BatchLaunch L;
            L.kind = BK_WAVE;
            L.op = op;
            L.grp = cur_grp;
            L.ct = kv.first.first;
            L.var = kv.first.second;
            L.njobs = static_cast<int>(kv.second.size());
            for (auto& w : kv.second) {
                L.work += static_cast<double>(w.g.I) * static_cast<double>(w.g.J);
                L.sel = std::max(L.sel, w.units);
                L.lds = std::max(L.lds, w.g.lds_bytes);
            }
            L.off = tw->put(kv.second);
            B->prog.push_back(L);
        }
        order_group(start);
    };
    auto add_reduce = [&](std::vector<rh::ReduceJob>& jobs) {
        if (jobs.empty()) return;
        BatchLaunch L;
        L.kind = BK_REDUCE;
        L.njobs = static_cast<int>(jobs.size());
        for (auto& j : jobs) L.sel = std::max(L.sel, j.I * j.K);
        L.off = tw->put(jobs);
        B->prog.push_back(L);
    };
    auto add_qr = [&](std::vector<rh::QrJob>& jobs) {
        ++cur_grp;
        const size_t start = B->prog.size();
        for (int ns = 1; ns <= 4; ++ns) {
            std::vector<rh::QrJob> sub;
            size_t lds = 0;
            for (auto& j : jobs)
                if ((j.K + 15) / 16 == ns) {
                    sub.push_back(j);
                    lds = std::max(lds, rh::hqr_lds_bytes(j.I, j.K));
                }
            if (sub.empty()) continue;
            BatchLaunch L;
            L.kind = BK_QR;
            L.grp = cur_grp;
            L.work = static_cast<double>(sub.size()) * ns;
            L.njobs = static_cast<int>(sub.size());
            L.sel = ns;
            L.lds = lds;
            L.off = tw->put(sub);
            B->prog.push_back(L);
        }
        order_group(start);
    };
    // report initialisation
    {
        std::vector<rh::ReportJob> jobs(n);
        for (int i = 0; i < n; ++i) {
            jobs[i] = rh::ReportJob{};
            jobs[i].rep = bufs[i].rep;
            jobs[i].order = N;
            for (int s = 0; s < N; ++s) {
                const Step& st = B->plans[i]->st[s];
                jobs[i].k_used[st.n] = st.capped ? -st.K : st.K;
            }
        }
        BatchLaunch L;
        L.kind = BK_INIT;
        L.njobs = n;
        L.off = tw->put(jobs);
        B->prog.push_back(L);
    }
    for (int s = 0; s < N; ++s) {
        // sketch, reduction, (norm of X), QR
        std::vector<PassJob> sj;
        std::vector<rh::ReduceJob> rj;
        std::vector<rh::QrJob> qj;
        std::vector<rh::SumJob> nj;
        for (int i = 0; i < n; ++i) {
            const Plan& pl = *B->plans[i];
            const Step& st = pl.st[s];
            const Buffers& b = bufs[i];
            PassJob j{&st.gs, rh::StreamArgs{}};
            j.a.src = cur[i];
            j.a.part_y = b.part;
            j.a.part_ss = s == 0 ? b.part_ss : nullptr;
            j.a.seed = pl.pr.seed;
            j.a.mode = static_cast<uint32_t>(st.n);
            j.a.tag = 2u;
            sj.push_back(j);
            rj.push_back(rh::ReduceJob{b.part, b.y, st.gs.grid, static_cast<int>(st.I), st.K,
                                       st.gs.I_pad, st.gs.K_pad});
            qj.push_back(rh::QrJob{b.y, b.q64, b.qT, static_cast<int>(st.I), st.K, B->dbl ? 1 : 0});
            if (s == 0) nj.push_back(rh::SumJob{b.part_ss, b.rep, st.gs.grid});
        }
        add_pass(rh::OP_SKETCH, sj);
        add_reduce(rj);
        if (s == 0) {
            BatchLaunch L;
            L.kind = BK_NORMX;
            L.njobs = n;
            L.off = tw->put(nj);
            B->prog.push_back(L);
        }
        add_qr(qj);
        // power steps (items with more power steps than it)
        for (int it = 0; it < B->maxq; ++it) {
            std::vector<PassJob> pj;
            std::vector<rh::ReduceJob> prj;
            std::vector<rh::QrJob> pqj;
            for (int i = 0; i < n; ++i) {
                const Plan& pl = *B->plans[i];
                if (pl.pr.q <= it) continue;
                const Step& st = pl.st[s];
                const Buffers& b = bufs[i];
                PassJob j{&st.gp, rh::StreamArgs{}};
                j.a.src = cur[i];
                j.a.mat = b.qT;
                j.a.part_y = b.part;
                pj.push_back(j);
                prj.push_back(rh::ReduceJob{b.part, b.y, st.gp.grid, static_cast<int>(st.I), st.K,
                                            st.gp.I_pad, st.gp.K_pad});
                pqj.push_back(rh::QrJob{b.y, b.q64, b.qT, static_cast<int>(st.I), st.K,
                                        B->dbl ? 1 : 0});
            }
            add_pass(rh::OP_POWER, pj);
            add_reduce(prj);
            add_qr(pqj);
        }
        // projection B = Q^T S_(n) with its Gram, the Gram reduction
        std::vector<PassJob> tj;
        std::vector<rh::ReduceJob> gj;
        std::vector<rh::EvdJob> ej;
        for (int i = 0; i < n; ++i) {
            const Plan& pl = *B->plans[i];
            const Step& st = pl.st[s];
            const Buffers& b = bufs[i];
            PassJob j{&st.gt, rh::StreamArgs{}};
            j.a.src = cur[i];
            j.a.mat = b.qT;
            j.a.out = b.B;
            j.a.part_g = b.part;
            tj.push_back(j);
            gj.push_back(rh::ReduceJob{b.part, b.C, st.gt.grid, st.K, st.K, st.gt.K_pad,
                                       st.gt.K_pad});
            rh::EvdJob e{};
            e.c = b.C;
            e.flags = &b.rep->flags;
            e.q = b.qT;
            e.u_out = B->factors[i][st.n];
            e.m_out = b.M;
            e.sigma = &b.rep->sigma[st.n][0];
            e.qwork = b.u64;
            e.K = st.K;
            e.I = static_cast<int>(st.I);
            e.R = st.R;
            e.use_v = 1;
            e.staged = rh::evd_factor_staged(st.K, st.I) ? 1 : 0;
            ej.push_back(e);
        }
        add_pass(rh::OP_TTM, tj);
        add_reduce(gj);
        ++cur_grp;
        const size_t evd_start = B->prog.size();
        for (int kb = 8; kb <= 64; kb += 8) {
            std::vector<rh::EvdJob> sub;
            size_t lds = 0;
            for (auto& e : ej)
                if (((e.K + 7) & ~7) == kb) {
                    sub.push_back(e);
                    lds = std::max(lds, rh::evd_factor_lds_bytes(e.K, e.I, e.staged != 0));
                }
            if (sub.empty()) continue;
            BatchLaunch L;
            L.kind = BK_EVD;
            L.grp = cur_grp;
            L.work = static_cast<double>(sub.size()) * kb;
            L.njobs = static_cast<int>(sub.size());
            L.sel = kb;
            L.lds = lds;
            L.off = tw->put(sub);
            B->prog.push_back(L);
        }
        order_group(evd_start);
        // truncation S <- Ubar_R^T B, written rotated
        std::vector<PassJob> rj2;
        for (int i = 0; i < n; ++i) {
            const Plan& pl = *B->plans[i];
            const Step& st = pl.st[s];
            const Buffers& b = bufs[i];
            void* dst = (s == N - 1) ? B->core[i] : ((s % 2 == 0) ? b.ping : b.pong);
            PassJob j{&st.gtr, rh::StreamArgs{}};
            j.a.src = b.B;
            j.a.mat = b.M;
            j.a.out = dst;
            j.a.out_t = 1;
            rj2.push_back(j);
            cur[i] = dst;
        }
        add_pass(rh::OP_TTM, rj2);
    }
    {
        std::vector<rh::FinishJob> fj(n);
        for (int i = 0; i < n; ++i)
            fj[i] = rh::FinishJob{B->core[i], bufs[i].rep, B->report[i], B->plans[i]->core_elems};
        BatchLaunch L;
        L.kind = BK_FINISH;
        L.njobs = n;
        L.off = tw->put(fj);
        B->prog.push_back(L);
    }
}

hipError_t launch_one(const rhosvd_batch* B, const BatchLaunch& L, hipStream_t s) {
    const void* t = B->ws + L.off;
    hipError_t e = hipSuccess;
    switch (L.kind) {
        case BK_STREAM:
            e = rh::launch_stream_batch(L.op, B->dbl, static_cast<const rh::StreamJob*>(t),
                                        L.njobs, L.sel, L.lds, s);
            break;
        case BK_REDUCE:
            e = rh::launch_reduce_parts_batch(B->dbl, static_cast<const rh::ReduceJob*>(t),
                                              L.njobs, L.sel, s);
            break;
        case BK_QR:
            e = rh::launch_hqr_batch(static_cast<const rh::QrJob*>(t), L.njobs, L.sel, L.lds, s);
            break;
        case BK_EVD:
            e = rh::launch_evd_factor_batch(B->dbl, static_cast<const rh::EvdJob*>(t), L.njobs,
                                            L.sel, L.lds, s);
            break;
        case BK_INIT:
            e = rh::launch_batch_report_init(static_cast<const rh::ReportJob*>(t), L.njobs, s);
            break;
        case BK_NORMX:
            e = rh::launch_batch_norm_x(static_cast<const rh::SumJob*>(t), L.njobs, s);
            break;
        case BK_FINISH:
            e = rh::launch_batch_finish(B->dbl, static_cast<const rh::FinishJob*>(t), L.njobs, s);
            break;
        case BK_WAVE:
            e = rh::launch_wave_batch(L.op, L.ct, L.var, static_cast<const rh::WaveJob*>(t),
                                      L.njobs, L.sel, L.lds, s);
            break;
        case BK_COL:
            e = rh::launch_col_batch(L.op, L.var, L.ct != 0, static_cast<const rh::ColJob*>(t),
                                     L.njobs, L.sel, L.lds, s);
            break;
        case BK_TRUNC:
            e = rh::launch_trunc_batch(B->dbl, L.ct, L.var, static_cast<const rh::TruncJob*>(t),
                                       L.njobs, L.sel, L.lds, s);
            break;
        default:
            e = hipErrorInvalidValue;
    }
    return e;
}

// Longest run of consecutive launches of one group.
size_t longest_group(const rhosvd_batch* B) {
    size_t best = 1;
    for (size_t i = 0; i < B->prog.size();) {
        size_t j = i + 1;
        while (j < B->prog.size() && B->prog[i].grp != 0 && B->prog[j].grp == B->prog[i].grp) ++j;
        best = std::max(best, j - i);
        i = j;
    }
    return best;
}

// The program on stream s.  With fork (the side streams and events exist),
// the largest launches of a group (up to kBatchBranches - 1) go to side
// streams that wait for s and that s waits for afterwards, and the others run
// one after another on s: captured, they are parallel branches of the graph,
// so one launch's tail overlaps the others.
hipError_t run_program(const rhosvd_batch* B, hipStream_t s, bool fork) {
    const size_t n = B->prog.size();
    for (size_t i = 0; i < n;) {
        size_t j = i + 1;
        while (j < n && B->prog[i].grp != 0 && B->prog[j].grp == B->prog[i].grp) ++j;
        hipError_t e = hipSuccess;
        // the group's largest launches (it is ordered by size) on side
        // branches, the rest one after another on s
        const size_t nside = std::min(j - i, kBatchBranches) - 1;
        if (fork && nside > 0 && nside <= B->side.size()) {
            e = hipEventRecord(B->fork, s);
            for (size_t k = 0; k < nside && e == hipSuccess; ++k) {
                hipStream_t t = B->side[k];
                e = hipStreamWaitEvent(t, B->fork, 0);
                if (e == hipSuccess) e = launch_one(B, B->prog[i + k], t);
                if (e == hipSuccess) e = hipEventRecord(B->joins[k], t);
            }
            for (size_t k = i + nside; k < j && e == hipSuccess; ++k) e = launch_one(B, B->prog[k], s);
            for (size_t k = 0; k < nside && e == hipSuccess; ++k)
                e = hipStreamWaitEvent(s, B->joins[k], 0);
        } else {
            for (size_t k = i; k < j && e == hipSuccess; ++k) e = launch_one(B, B->prog[k], s);
        }
        if (e != hipSuccess) return e;
        i = j;
    }
    return hipSuccess;
}

// Upper bound of the tables: every launch holds at most one job per item.
size_t tables_bound(int n, int N, int maxq) {
    const size_t per_item_jobs = static_cast<size_t>(N) * (7 + 3 * maxq) + 3;
    // a pass may split into one tiled launch, five wave launches per compute
    // type and ten column-kernel launches (shape x flag)
    const size_t job = std::max({sizeof(rh::StreamJob), sizeof(rh::WaveJob), sizeof(rh::ColJob)});
    return (per_item_jobs * n * job + 256 * (N * (12 + 8 * maxq) * 20 + 8) + 4095) &
           ~static_cast<size_t>(4095);
}

// Mode-1 sketch of every item with the tile width cap `cmax` and `tpu` tiles
// per workgroup: the time of the fastest of three launches (ms).
int32_t time_candidate(rhosvd_batch* B, int cmax, int tpu, hipStream_t s, float* ms) {
    std::vector<rh::StreamJob> jobs;
    size_t lds = 0;
    int maxu = 1;
    for (int i = 0; i < B->n; ++i) {
        Plan pl = *B->plans[i];
        batch_geometry(&pl, cmax, tpu);
        Buffers b;
        carve(pl, B->ws + B->region[i], &b);
        const Step& st = pl.st[0];
        if (st.gs.kind != PASS_TILED) continue;       // the wave kernels take no tile parameters
        rh::StreamJob j{};
        j.g = st.gs.sg;
        j.units = st.gs.grid;
        j.a.src = B->x[i];
        j.a.part_y = b.part;
        j.a.seed = pl.pr.seed;
        j.a.mode = static_cast<uint32_t>(st.n);
        j.a.tag = 2u;
        jobs.push_back(j);
        lds = std::max(lds, j.g.lds_bytes);
        maxu = std::max(maxu, j.units);
    }
    if (jobs.empty()) {
        *ms = 0.0f;
        return RHOSVD_OK;
    }
    RH_HIP(hipMemcpy(B->ws, jobs.data(), jobs.size() * sizeof(rh::StreamJob), hipMemcpyHostToDevice));
    hipEvent_t e0, e1;
    RH_HIP(hipEventCreate(&e0));
    RH_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    for (int r = 0; r < 3; ++r) {
        RH_HIP(hipEventRecord(e0, s));
        RH_HIP(rh::launch_stream_batch(rh::OP_SKETCH, B->dbl,
                                       reinterpret_cast<const rh::StreamJob*>(B->ws),
                                       static_cast<int>(jobs.size()), maxu, lds, s));
        RH_HIP(hipEventRecord(e1, s));
        RH_HIP(hipEventSynchronize(e1));
        float t = 0.0f;
        RH_HIP(hipEventElapsedTime(&t, e0, e1));
        if (r > 0 && t < best) best = t;     // the first launch warms up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = best;
    return RHOSVD_OK;
}

}  // namespace

extern "C" {

int32_t rhosvd_batch_create(rhosvd_ctx* ctx, int32_t count, const rhosvd_tensor* x,
                            const rhosvd_params* p, const rhosvd_output* out,
                            rhosvd_batch** batch, size_t* ws_bytes) {
    if (!ctx || count < 1 || !x || !p || !out || !batch || !ws_bytes) return RHOSVD_EINVAL;
    *batch = nullptr;
    rhosvd_batch* B = new (std::nothrow) rhosvd_batch;
    if (!B) return RHOSVD_ENOMEM;
    B->ctx = ctx;
    B->n = count;
    int32_t rc = RHOSVD_OK;
    size_t off = 0;
    for (int i = 0; i < count && rc == RHOSVD_OK; ++i) {
        Problem pr;
        rc = validate(&x[i], &p[i], &pr, true);
        if (rc != RHOSVD_OK) break;
        if (pr.algo != RHOSVD_R_STHOSVD || (pr.explicit_error)) { rc = RHOSVD_EUNSUPPORTED; break; }
        if (!out[i].core || !out[i].factors) { rc = RHOSVD_EINVAL; break; }
        for (int nn = 0; nn < pr.N; ++nn)
            if (!out[i].factors[nn]) rc = RHOSVD_EINVAL;
        if (rc != RHOSVD_OK) break;
        if (i == 0) {
            B->N = pr.N;
            B->dbl = pr.dbl;
        } else if (pr.N != B->N || pr.dbl != B->dbl) {
            rc = RHOSVD_EUNSUPPORTED;
            break;
        }
        pr.kernels = RHOSVD_KERNELS_TILED;
        Plan* pl = new (std::nothrow) Plan;
        if (!pl) { rc = RHOSVD_ENOMEM; break; }
        B->plans.push_back(pl);
        rc = build_plan(pr, 256, pl);
        if (rc != RHOSVD_OK) break;
        if (!pl->rotated) { rc = RHOSVD_EUNSUPPORTED; break; }
        for (int s = 0; s < pr.N; ++s)
            if (pl->st[s].I > 256 || pl->st[s].K > 64) rc = RHOSVD_EUNSUPPORTED;
        if (rc != RHOSVD_OK) break;
        // the region holds the partials of up to kBatchUnits workgroups per pass
        batch_geometry(pl, 64, 1);
        pl->part_bytes = 0;
        pl->max_grid = kBatchUnits;
        for (int s = 0; s < pr.N; ++s) {
            const Step& st = pl->st[s];
            const Pass* ps[4] = {&st.gs, &st.gp, &st.gt, &st.gtr};
            for (const Pass* q : ps) {
                const size_t big = static_cast<size_t>(std::max(q->I_pad, q->K_pad));
                const size_t b = static_cast<size_t>(kBatchUnits) * q->K_pad * big * pr.elem;
                pl->part_bytes = std::max(pl->part_bytes, b);
            }
        }
        B->maxq = std::max(B->maxq, pr.q);
        B->x.push_back(x[i].data);
        B->core.push_back(out[i].core);
        B->report.push_back(out[i].report);
        B->factors.emplace_back(out[i].factors, out[i].factors + pr.N);
        Buffers b;
        const size_t sz = (carve(*pl, nullptr, &b) + 4095) & ~static_cast<size_t>(4095);
        B->region.push_back(off);
        off += sz;
    }
    if (rc != RHOSVD_OK) {
        delete B;
        return rc;
    }
    B->tables_cap = tables_bound(count, B->N, B->maxq);
    for (auto& r : B->region) r += B->tables_cap;
    B->ws_bytes = B->tables_cap + off;
    *ws_bytes = B->ws_bytes;
    *batch = B;
    return RHOSVD_OK;
}

int32_t rhosvd_batch_bind(rhosvd_batch* B, void* workspace, size_t ws_bytes, int32_t autotune,
                          void* stream) {
    if (!B || !workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return RHOSVD_EINVAL;
    if (ws_bytes < B->ws_bytes) return RHOSVD_ENOMEM;
    B->ws = static_cast<unsigned char*>(workspace);
    if (B->exec) {
        (void)hipGraphExecDestroy(B->exec);
        B->exec = nullptr;
    }
    if (B->graph) {
        (void)hipGraphDestroy(B->graph);
        B->graph = nullptr;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    rhosvd_ctx* ctx = B->ctx;
    if (!ctx->tuned && autotune) {
        // tile width cap x tiles per workgroup, timed on this batch's mode-1
        // sketch; the choice is kept in the context so that every later batch
        // (and a batch of one) computes with the same tiles
        const int cm[3] = {64, 32, 16}, tp[4] = {1, 2, 4, 8};
        float best = 1e30f;
        int bc = 64, bt = 1;
        for (int c : cm)
            for (int t : tp) {
                float ms = 0.0f;
                const int32_t rc = time_candidate(B, c, t, s, &ms);
                if (rc != RHOSVD_OK) return rc;
                if (ms < best) {
                    best = ms;
                    bc = c;
                    bt = t;
                }
            }
        ctx->tuned = 1;
        ctx->tune_cmax = bc;
        ctx->tune_tpu = bt;
        ctx->tune_ms = best;
    }
    const int cmax = ctx->tuned ? ctx->tune_cmax : 64;
    const int tpu = ctx->tuned ? ctx->tune_tpu : 1;
    for (Plan* pl : B->plans) batch_geometry(pl, cmax, tpu);
    TableWriter tw;
    build_program(B, &tw);
    if (tw.bytes.size() > B->tables_cap) return RHOSVD_ENOMEM;
    RH_HIP(hipMemcpy(B->ws, tw.bytes.data(), tw.bytes.size(), hipMemcpyHostToDevice));
    return RHOSVD_OK;
}

int32_t rhosvd_batch_run(rhosvd_batch* B, int32_t use_graph, void* stream) {
    if (!B || !B->ws) return RHOSVD_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = -1;
    RH_HIP(hipGetDevice(&dev));
    if (dev != B->ctx->device) RH_HIP(hipSetDevice(B->ctx->device));
    hipError_t e = hipSuccess;
    if (!use_graph || !s) {
        e = run_program(B, s, false);
    } else {
        if (!B->exec) {
            // side streams and events for the longest group, made before the capture
            const size_t need = std::min(longest_group(B), kBatchBranches) - 1;
            while (e == hipSuccess && B->side.size() < need) {
                hipStream_t t = nullptr;
                e = hipStreamCreateWithFlags(&t, hipStreamNonBlocking);
                if (e == hipSuccess) B->side.push_back(t);
            }
            while (e == hipSuccess && B->joins.size() < need) {
                hipEvent_t ev = nullptr;
                e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
                if (e == hipSuccess) B->joins.push_back(ev);
            }
            if (e == hipSuccess && !B->fork) e = hipEventCreateWithFlags(&B->fork, hipEventDisableTiming);
            if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t er = run_program(B, s, true);
                hipGraph_t g = nullptr;
                e = hipStreamEndCapture(s, &g);
                if (er != hipSuccess) e = er;
                if (e == hipSuccess) {
                    B->graph = g;
                    e = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
                } else if (g) {
                    (void)hipGraphDestroy(g);
                }
            }
        }
        if (e == hipSuccess) e = hipGraphLaunch(B->exec, s);
    }
    if (dev != B->ctx->device) (void)hipSetDevice(dev);
    if (e != hipSuccess) return hip_fail(e);
    return RHOSVD_OK;
}

void rhosvd_batch_destroy(rhosvd_batch* B) { delete B; }

int32_t rhosvd_batch_launches(const rhosvd_batch* B) {
    return B ? static_cast<int32_t>(B->prog.size()) : 0;
}

}  // extern "C"
