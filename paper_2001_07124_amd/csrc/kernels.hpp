// Host-side interface of the kernels (launchers).  Every launcher enqueues on
// `stream` and returns the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rhosvd.h"

namespace rh {

enum StreamOp { OP_SKETCH = 0, OP_POWER = 1, OP_TTM = 2 };

// Geometry of one streaming pass over an n-unfolding view (L, I, T) of a
// first-index-fastest tensor: element (i, j = l + L t) at src[l + L (i + I t)].
struct StreamGeom {
    int64_t L, I, T, J;   // J = L T
    int K;                // sketch width (SKETCH/POWER) or output rows Kout (TTM)
    int I_pad, K_pad;     // rounded up to 16
    int P;                // LDS pitch of the tile (>= I_pad)
    int KW;               // LDS pitch of the K-wide operands (>= K_pad)
    int C;                // unfolding columns per tile (16, 32 or 64)
    int64_t ntiles;
    int grid;             // workgroups (each walks tiles grid-stride)
    size_t lds_bytes;
};

// Structured test matrix of Section 5.1 (the Khatri-Rao form): the
// unfolding column j, split in mixed radix over ext[0 .. nq) (fastest first:
// the other modes in the order they are stored), gives
// Omega(j, k) = prod_q tab_q(i_q, k), each tab_q ext[q] x K column-major in
// the tensor's dtype.  nq = 0 selects the Gaussian stream.  Rows past J and
// columns past K (the padding of the kernels' tiles) read as row J - 1 and
// column K - 1 so that no table is read out of range; their products meet
// zero data or land in dropped outputs.
struct KrArgs {
    const void* tab[RHOSVD_MAX_ORDER - 1];
    int ext[RHOSVD_MAX_ORDER - 1];
    int nq;
    int K;
    int64_t J;
};

template <typename V>
__device__ __forceinline__ V kr_entry(const KrArgs& kr, int64_t j, int k) {
    uint32_t jj = static_cast<uint32_t>(j < kr.J ? j : kr.J - 1);
    const size_t kk = static_cast<size_t>(k < kr.K ? k : kr.K - 1);
    V w = V(1);
    for (int q = 0; q < kr.nq; ++q) {
        const uint32_t e = static_cast<uint32_t>(kr.ext[q]);
        const uint32_t nx = jj / e;
        w *= static_cast<const V*>(kr.tab[q])[(jj - nx * e) + kk * e];
        jj = nx;
    }
    return w;
}

// Rows j0 .. j0 + 3 of column k: the slower digits' product once, the
// fastest digit per row (the full product where it wraps).
template <typename V>
__device__ __forceinline__ void kr_entry4(const KrArgs& kr, int64_t j0, int k, V (&w)[4]) {
    const int64_t jl = kr.J - 1;
    const uint32_t e0 = static_cast<uint32_t>(kr.ext[0]);
    const size_t kk = static_cast<size_t>(k < kr.K ? k : kr.K - 1);
    const uint32_t jj = static_cast<uint32_t>(j0 < jl ? j0 : jl);
    uint32_t r = jj / e0;
    const uint32_t i0 = jj - r * e0;
    V rest = V(1);
    for (int q = 1; q < kr.nq; ++q) {
        const uint32_t e = static_cast<uint32_t>(kr.ext[q]);
        const uint32_t nx = r / e;
        rest *= static_cast<const V*>(kr.tab[q])[(r - nx * e) + kk * e];
        r = nx;
    }
    const V* t0 = static_cast<const V*>(kr.tab[0]) + kk * e0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        w[e] = (i0 + e < e0 && j0 + e <= jl) ? rest * t0[i0 + e] : kr_entry<V>(kr, j0 + e, k);
}

struct StreamArgs {
    const void* src;
    const void* mat;      // POWER: Q (I x K); TTM: M (I x Kout); column-major
    void* out;            // TTM: folded output
    void* part_y;         // [grid][K_pad][I_pad] partial sketches (SKETCH/POWER)
    void* part_g;         // [grid][K_pad][K_pad] partial Gram (TTM, optional)
    double* part_ss;      // [grid] partial sum of squares of src (optional)
    uint64_t seed;
    uint32_t mode, tag;
    int out_t;            // TTM with L == 1: write out[r * J + j] (modes rotated) instead of out[j * K + r]
    KrArgs kr;            // SKETCH: the structured test matrix when kr.nq > 0
};

// Plan the geometry of a pass; returns false if the shape exceeds the
// implemented limits.  elem = sizeof(float) or sizeof(double).
bool plan_stream(int op, int elem, int64_t L, int64_t I, int64_t T, int K, int num_cu,
                 StreamGeom* g, int cmax = 64);

hipError_t launch_stream(int op, bool dbl, const StreamGeom& g, const StreamArgs& a,
                         hipStream_t s);

// One pass of many independent problems in one launch (device table of
// jobs): job y runs on `units` workgroups (grid x = the largest units),
// partial slots 0 .. units - 1 of its own buffers.  lds: the largest of the
// jobs' g.lds_bytes.
struct StreamJob {
    StreamGeom g;
    StreamArgs a;
    int units;
    int pad_;
};
hipError_t launch_stream_batch(int op, bool dbl, const StreamJob* jobs, int njobs, int max_units,
                               size_t lds, hipStream_t s);

// Matrix-core input precision of the wave-private FP32 kernels.
enum CompType { CT_F32 = 0, CT_BF16 = 1, CT_BF16X3 = 2, CT_BF16X2 = 3, CT_FP8 = 4 };

// Geometry of a wave-private pass (kernels_wave.hip): each wave owns blocks
// of 16 unfolding columns; IB = ceil(I / 16) row blocks, NB = ceil(K / 16)
// column blocks of the K-wide operand.
struct WGeom {
    int64_t L, I, T, J;
    int K, IB, NB, ct, variant;
    size_t q_bytes, scr_bytes, lds_bytes;
    int64_t nblocks;
    int grid;
    int vec4;             // L == 1 and I % 4 == 0: 16-byte row loads
    int rs;               // waves sharing a column block (1, or 4 for tall modes)
    int IBW;              // row blocks per wave when rs > 1
    size_t xr_off;        // rs > 1: offset of the cross-wave exchange of Z
};

bool plan_wave(int op, int ct, int64_t L, int64_t I, int64_t T, int K, int num_cu, WGeom* g);
hipError_t launch_wave(int op, const WGeom& g, const StreamArgs& a, hipStream_t s);

// One wave-kernel pass of many problems in one launch (device table): job y
// runs on `units` workgroups of grid x (partial slots 0 .. units - 1).  The
// batch instantiations are the generic row-block x operand-block bounds of
// wave_batch_variant (a geometry with another variant is not batched).
struct WaveJob {
    WGeom g;
    StreamArgs a;
    int units;
    int want_ss;
    int want_gram;
    int pad_;
};
int wave_batch_variant(const WGeom& g);   // 0..3, or -1
bool wave_batch_ct(int op, int ct);       // the compute type has batched instantiations
hipError_t launch_wave_batch(int op, int ct, int variant, const WaveJob* jobs, int njobs,
                             int max_units, size_t lds, hipStream_t s);

// Geometry of a column-block pass (kernels_col.hip): contiguous unfolding
// (L = 1), bf16 matrix cores, blocks of 32 columns, nch 32-row chunks and nb
// 16-column blocks of the K-wide operand.  Sketch: CT_BF16; power step and
// mode-n product: CT_BF16X2 or CT_BF16X3.
struct ColGeom {
    int64_t I, J;
    int K, nch, nb, variant, rowp;
    int split;            // the tensor split into hi + lo bf16 in Z = S^T M (CT_BF16X3)
    int fp8;              // the sketch on e4m3 inputs (CT_FP8)
    int red3;             // LDS holds three waves' Y accumulators for the final reduction
    size_t mfr_bytes, lds_bytes;
    int64_t nblocks;
    int grid, I_pad, K_pad;
};

bool plan_col(int op, int ct, int64_t L, int64_t I, int64_t T, int K, int num_cu, ColGeom* g);
hipError_t launch_col(int op, const ColGeom& g, const StreamArgs& a, hipStream_t s);

// The column kernels over a batch: job y on workgroups 0 .. units - 1 of
// grid x.  plan_col_batch plans a contiguous unfolding (L = 1) on one of the
// batched shapes (g->variant indexes them); the bf16 sketch and the split
// power step / mode-n product only.  flag: the sketch's sum of squares, or
// the mode-n product's Gram.
struct ColJob {
    ColGeom g;
    StreamArgs a;
    int units;
    int pad_;
};
bool plan_col_batch(int op, int ct, int64_t I, int64_t T, int K, ColGeom* g);
hipError_t launch_col_batch(int op, int shape, bool flag, const ColJob* jobs, int njobs, int max_units,
                            size_t lds, hipStream_t s);

// Truncation in the rotated layout (kernels_trunc.hip): out[r J + j] =
// sum_k M(k, r) B(k, j) for B K x J and M K x R column-major, K <= 64 (32
// for FP64), in the tensor's precision with one column per lane.
struct TruncGeom {
    int K, R, rb, grid;          // rb: row tiles of 16 outputs
    int64_t J;
    size_t lds_bytes;
};
// the rotated truncation kernel's geometry (K = I rows of B, R outputs, T
// columns); false when it does not take the shape or, unless any_size, when
// the column kernels are faster there
bool plan_trunc(bool dbl, int64_t I, int64_t T, int R, int num_cu, bool any_size, TruncGeom* g);
hipError_t launch_trunc(bool dbl, const TruncGeom& g, const void* B, const void* M, void* out,
                        hipStream_t s);
// Many truncations in one launch: job y on workgroups 0 .. units - 1 of
// grid x; every job of a launch has (R + 15) / 16 = rt and trunc_kqm(K) = kqm;
// lds: the largest trunc lds_bytes among them.
struct TruncJob {
    const void* b;
    const void* m;
    void* out;
    int K, R;
    int64_t J;
    int units;
    int pad_;
};
int trunc_kqm(int K);
size_t trunc_lds_bytes(int K, bool dbl);
hipError_t launch_trunc_batch(bool dbl, int rt, int kqm, const TruncJob* jobs, int njobs, int max_units,
                              size_t lds, hipStream_t s);

// Fixed-order reductions of per-workgroup partials.
hipError_t launch_reduce_y(bool dbl, const void* part, int G, int I, int K, int I_pad, int K_pad,
                           double* y, hipStream_t s);
hipError_t launch_reduce_ss(const double* part, int G, double* out, hipStream_t s);

// CholeskyQR2 (shifted CholeskyQR3 when needed, Householder fallback).  y is
// I x K double; q64 points at 2 I K doubles (Q in FP64, then scratch); q_out
// receives Q in the tensor's precision.  Y is staged in LDS when it fits
// (kernels_small.hip), else the global-memory kernel (kernels.hip) runs.
hipError_t launch_cqr(const double* y, int64_t I, int K, bool dbl, void* q_out, double* q64,
                      uint32_t* flags, hipStream_t s);
hipError_t launch_cqr_lds(const double* y, int64_t I, int K, bool dbl, void* q_out, double* q64,
                          uint32_t* flags, hipStream_t s);
hipError_t launch_cqr_global(const double* y, int64_t I, int K, bool dbl, void* q_out,
                             double* q64, uint32_t* flags, hipStream_t s);
size_t cqr_lds_bytes(int64_t I, int K);
// R-PET core recovery operator: pt = (pinv(Omt^T Q))^T (S x K column-major)
// for Omt (I x S) and Q (I x K), in FP64 arithmetic (kernels_small.hip).
hipError_t launch_lsq_pinv(bool dbl, const void* omt, const void* q, int I, int S, int K, void* pt,
                           uint32_t* flags, hipStream_t s);

// Symmetric EVD of the K x K Gram C (FP64, sorted descending) followed, in
// the same launch, by the factor step: U = Q V[:, :R] (identity V when
// use_v == 0), canonical signs, M = V_R (K x R, same signs), sigma =
// sqrt(max(lambda, 0))[:R].  u64: evd_qwork_doubles(K, I) doubles of scratch
// for Q when it does not fit in LDS.  flags receives RHOSVD_FLAG_EVD_NOCONV
// when the eigenpairs fail the residual / orthogonality check.
hipError_t launch_evd_factor(bool dbl, const double* c, int K, uint32_t* flags, const void* q,
                             int64_t I, int R, int use_v, void* u_out, void* m_out, double* sigma,
                             double* u64, hipStream_t s);
// The EVD alone: v (K x K), lambda (K), descending.
hipError_t launch_evd(const double* c, int K, double* v, double* lambda, uint32_t* flags,
                      hipStream_t s);
size_t evd_qwork_doubles(int K, int64_t I);
hipError_t launch_reduce_parts(bool dbl, const void* part, int G, int I, int K, int I_pad,
                               int K_pad, double* y, hipStream_t s);

hipError_t launch_sumsq(bool dbl, const void* x, int64_t n, double* part, int G, hipStream_t s);

hipError_t launch_omega_fill(bool dbl, uint64_t seed, int mode, int tag, int64_t J, int K,
                             void* out, hipStream_t s);

// Up to kMax Gaussian tables (stream (seed, word, tag), J x K column-major
// each, as launch_omega_fill) in one launch.
struct KrFill {
    static constexpr int kMax = 48;
    struct Table {
        void* out;
        int64_t J;
        int K;
        uint32_t word;
    } t[kMax];
    int count;
    uint32_t tag;
    uint64_t seed;
};
hipError_t launch_kr_fill(bool dbl, const KrFill& f, hipStream_t s);

hipError_t launch_gram_reduce(bool dbl, const void* part, int G, int K, int K_pad, double* c,
                              hipStream_t s);

// Single-pass sketch of every mode (kernels_allmode.hip): Y_n = X_(n) Omega_n
// (tag `tag`, cyclic rows) for all n from one read of X, plus per-workgroup
// sums of squares.  part: grid x S partials in X's dtype; the reduce writes
// all Y_n into y (S doubles; Y_n at yoff[n], I_n x K_n column-major).
struct AllModeArgs {
    const void* x;
    void* part;
    double* part_ss;          // grid doubles, or null
    uint64_t seed;
    uint32_t tag;
    int N, KMAX, grid;
    int64_t dims[RHOSVD_MAX_ORDER];
    int K[RHOSVD_MAX_ORDER];
    int b[RHOSVD_MAX_ORDER];          // tile extents
    int64_t bs[RHOSVD_MAX_ORDER];     // tile strides (first fastest)
    int64_t ntile[RHOSVD_MAX_ORDER];  // tiles along each mode
    int64_t xs[RHOSVD_MAX_ORDER];     // strides of X
    int64_t yoff[RHOSVD_MAX_ORDER];   // offset of Y_n in a partial / in y
    int64_t J[RHOSVD_MAX_ORDER], T[RHOSVD_MAX_ORDER];
    int64_t TB, S, ntiles;
    size_t lds_bytes;
};
bool plan_allmode(int N, const int64_t* dims, const int* K, int num_cu, int elem, AllModeArgs* a);
hipError_t launch_allmode(bool dbl, const AllModeArgs& a, hipStream_t s);
hipError_t launch_allmode_reduce(bool dbl, const AllModeArgs& a, double* y, hipStream_t s);

// Device tables of the batched small kernels (one problem per job).
struct ReduceJob {          // y = sum of G partials [G][K_pad][I_pad] of an I x K result
    const void* part;
    double* y;
    int G, I, K, I_pad, K_pad;
};
struct QrJob {              // Householder QR of Y (I x K, I <= 256, K <= 64)
    const double* y;
    double* q64;
    void* q_out;
    int I, K, dbl;
};
struct EvdJob {             // EVD of the K x K Gram c followed by the factor step
    const double* c;
    uint32_t* flags;
    const void* q;
    void* u_out;
    void* m_out;
    double* sigma;
    double* qwork;
    int K, I, R, use_v, staged;
};
struct ReportJob {          // report initialisation of one item
    rhosvd_report* rep;
    int order;
    int k_used[RHOSVD_MAX_ORDER];   // negative: capped
};
struct SumJob {             // rep->norm_x2 = sum of G per-workgroup sums
    const double* part;
    rhosvd_report* rep;
    int G;
};
struct FinishJob {          // rep->norm_core2 = ||core||^2, then rep copied to out_report
    const void* core;
    rhosvd_report* rep;
    void* out_report;
    int64_t core_elems;
};
hipError_t launch_reduce_parts_batch(bool dbl, const ReduceJob* jobs, int njobs, int max_elems,
                                     hipStream_t s);
hipError_t launch_batch_report_init(const ReportJob* jobs, int njobs, hipStream_t s);
hipError_t launch_batch_norm_x(const SumJob* jobs, int njobs, hipStream_t s);
hipError_t launch_batch_finish(bool dbl, const FinishJob* jobs, int njobs, hipStream_t s);
hipError_t launch_hqr_batch(const QrJob* jobs, int njobs, int ns, size_t lds, hipStream_t s);
size_t hqr_lds_bytes(int I, int K);
bool evd_factor_staged(int K, int64_t I);
size_t evd_factor_lds_bytes(int K, int64_t I, bool staged);
hipError_t launch_evd_factor_batch(bool dbl, const EvdJob* jobs, int njobs, int kb, size_t lds,
                                   hipStream_t s);

// Explicit residual ||X - G x_1 U_1 ... x_N U_N||^2 (kernels_resid.hip).
// gate: one device int written by launch_resid_gate (1 when requested or when
// the report's identity-based E is below 1e-2); every other launch returns
// at once when it is 0.  launch_expand: out = in x_n U for the view (L, R, T)
// of `in` and U (I x R, column-major), out viewed (L, I, T).  launch_resid:
// X viewed (M, IN), W (M x R), U_N (IN x R) column-major; part holds
// kResidGrid doubles; the sum lands in report->resid2 with
// RHOSVD_FLAG_E_EXPLICIT set.
constexpr int kResidGrid = 2048;
hipError_t launch_resid_gate(void* rep, int requested, int* gate, hipStream_t s);
hipError_t launch_expand(bool dbl, const int* gate, const void* in, const void* u, int64_t L,
                         int I, int R, int64_t T, void* out, hipStream_t s);
hipError_t launch_resid(bool dbl, const int* gate, const void* x, const void* w, const void* un,
                        int64_t M, int IN, int R, double* part, void* rep, hipStream_t s);

struct ReportInit {
    int32_t order;
    int32_t k_used[16];
};
hipError_t launch_report_init(void* rep, ReportInit ri, hipStream_t s);
// After mode n of the fixed-precision path: k_used[n] = |k| (k < 0 marks a
// capped sketch width, which also sets the flag) and sigma[n][r ..] = 0.
hipError_t launch_report_mode(void* rep, int n, int k, int r, hipStream_t s);
hipError_t launch_copy_bytes(const void* src, void* dst, size_t n, hipStream_t s);

}  // namespace rh
