// Small dense steps between the streaming passes, written for latency:
//   k_reduce_parts  fixed-order sum of per-workgroup partials (many workgroups)
//   k_cqr           CholeskyQR2 of Y (I x K) with Y resident in LDS: Gram and
//                   triangular update on the f64 matrix cores, the K x K
//                   Cholesky factor and its inverse in one wave's registers
//                   (Algorithm 1 step 3)
//   k_evd_factor    Jacobi EVD of the K x K Gram (Algorithm 1 step 5) fused
//                   with U = Q V[:, :R], sign canonicalisation, M = V_R diag(s)
//                   and sigma (steps 6-7)
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "householder.hpp"
#include "kernels.hpp"
#include "rhosvd.h"

namespace rh {

// ---------------------------------------------------------------------------
// out[e] = sum_g part[g * stride + off(e)], e < I K, fixed order in g.
// Block: 64 elements x 4 partial groups; group q sums g = q, q + 4, ...
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_reduce_parts(const T* __restrict__ part, int G, int I,
                                                         int K, int I_pad, int K_pad,
                                                         double* __restrict__ y) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (e < I * K) {
        const int k = e / I, i = e - k * I;
        const size_t stride = static_cast<size_t>(K_pad) * I_pad;
        const T* p = part + static_cast<size_t>(k) * I_pad + i;
        for (int g = q; g < G; g += 4) s += static_cast<double>(p[g * stride]);
    }
    red[q][lane] = s;
    __syncthreads();
    if (q == 0 && e < I * K) y[e] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

hipError_t launch_reduce_parts(bool dbl, const void* part, int G, int I, int K, int I_pad,
                               int K_pad, double* y, hipStream_t s) {
    const dim3 grid((I * K + 63) / 64);
    if (dbl)
        hipLaunchKernelGGL(k_reduce_parts<double>, grid, dim3(kBlock), 0, s,
                           static_cast<const double*>(part), G, I, K, I_pad, K_pad, y);
    else
        hipLaunchKernelGGL(k_reduce_parts<float>, grid, dim3(kBlock), 0, s,
                           static_cast<const float*>(part), G, I, K, I_pad, K_pad, y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CholeskyQR2 with W = Y resident in LDS, zero-padded to I16 = 16 ceil(I/16)
// rows and KP16 = 16 ceil(K/16) columns (row pitch P = KP16 + 1):
//   G = W^T W               f64 matrix cores, all waves
//   G = L L^T, X = L^{-1}   one wave; lane i keeps row i of G, L, X in registers
//   W <- W X^T              f64 matrix cores; each wave owns 16-row blocks
// twice, three times after a shift.  KB (a multiple of 8, >= K) is the length
// of the register rows; X is zero outside its K x K block, so the padding of
// W stays zero.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
}

__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b), l));
    const unsigned hi =
        static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), l));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

struct CqrGeom {
    int I, K, I16, KP16, P;
};

// G (pitch KP16, K x K block written) = W^T W + shift I; diag0 = diag(G).
// Wave w forms the tiles w, w + 4, ... of the upper block triangle with two
// interleaved accumulator chains; the mirrored tile is written from the same
// registers.
__device__ void mfma_gram(const double* W, const CqrGeom g, double* G, double shift,
                                       double* diag0) {
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int m = lane & 15, kq = lane >> 4;
    const int nt = g.KP16 >> 4;
    const int npair = nt * (nt + 1) / 2;
    for (int t = wave; t < npair; t += kBlock / kWave) {
        int ta = 0, rem = t;
        while (rem >= nt - ta) {
            rem -= nt - ta;
            ++ta;
        }
        const int tb = ta + rem;
        const double* wa = W + kq * g.P + 16 * ta + m;
        const double* wb = W + kq * g.P + 16 * tb + m;
        f64x4 acc0 = zero4<f64x4>(), acc1 = zero4<f64x4>();
        for (int i0 = 0; i0 < g.I16; i0 += 8) {
            const double a0 = wa[i0 * g.P], b0 = wb[i0 * g.P];
            const double a1 = wa[(i0 + 4) * g.P], b1 = wb[(i0 + 4) * g.P];
            acc0 = Mma<double>::step(a0, b0, acc0);
            acc1 = Mma<double>::step(a1, b1, acc1);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * ta + Mma<double>::row(kq, r), col = 16 * tb + m;
            if (row < g.K && col < g.K) {
                const double x = (acc0[r] + acc1[r]) + (row == col ? shift : 0.0);
                G[row * g.KP16 + col] = x;
                G[col * g.KP16 + row] = x;
                if (row == col) diag0[row] = x;
            }
        }
    }
}

// One wave.  Right-looking Cholesky G = L L^T with lane i holding row i:
// step j takes the pivot from lane j, L(j+1, j) by a lane read (the next
// pivot depends on nothing else), and the rest of column j through S.  Then
// X = L^{-1} by rows, lane i solving x L = e_i from the last column down with
// the rows of L broadcast from S.  S may alias G (read into registers first).
// Out: X (pitch XP; rows >= K zero).  Returns false, uniformly, on a pivot not
// above 1e-14 of its original diagonal.
template <int KB>
__device__ bool wave_chol_inv(const double* G, const double* diag0, double* S, double* X, int K,
                              int XP) {
    const int lane = threadIdx.x & 63;
    const int li = lane < KB ? lane : KB - 1;
    double g[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) g[c] = (li < K && c < K) ? G[li * XP + c] : (li == c ? 1.0 : 0.0);
    const double dgl = (li < K) ? diag0[li] : 1.0;
    double dinvl = 0.0;     // lane j: 1 / L(j, j)
    bool ok = true;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        if (j < K && ok) {
            const double d = readlane_d(g[j], j);
            const double d0 = readlane_d(dgl, j);
            if (!(d > 1e-14 * d0) || !(d0 > 0.0)) {
                ok = false;
            } else {
                const double inv = rsqrt(d);
                const double r = d * inv;
                const double l = (li > j) ? g[j] * inv : (li == j ? r : 0.0);
                if (li == j) dinvl = inv;
                g[j] = l;
                if (j + 1 < KB) g[j + 1] = fma(-l, readlane_d(l, j + 1), g[j + 1]);
                if (j + 2 < KB) {
                    if (lane < KB) S[j * XP + lane] = l;
#pragma unroll
                    for (int c = j + 2; c < KB; ++c) g[c] = fma(-l, S[j * XP + c], g[c]);
                }
            }
        }
    }
    if (!ok) return false;
    if (lane < KB) {
#pragma unroll
        for (int c = 0; c < KB; ++c) S[lane * XP + c] = g[c];
    }
    double acc[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) acc[k] = 0.0;
#pragma unroll
    for (int m = KB - 1; m >= 0; --m) {
        if (m < K) {
            const double x = ((li == m ? 1.0 : 0.0) - acc[m]) * readlane_d(dinvl, m);
            acc[m] = x;
#pragma unroll
            for (int k = 0; k < m; ++k) acc[k] = fma(x, S[m * XP + k], acc[k]);
        } else {
            acc[m] = 0.0;
        }
    }
    if (lane < KB && li < K) {
#pragma unroll
        for (int c = 0; c < KB; ++c) X[lane * XP + c] = acc[c];
    }
    return true;
}

// W <- W X^T with X lower triangular (pitch KP16).  Wave w owns the 16-row
// blocks w, w + 4, ...; the up to four column tiles of a block share the A
// operand and are finished in registers before the block is overwritten.
__device__ void mfma_apply(double* W, const CqrGeom g, const double* X) {
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int m = lane & 15, kq = lane >> 4;
    const int nt = g.KP16 >> 4;
    const int nrb = g.I16 >> 4;
    for (int rb = wave; rb < nrb; rb += kBlock / kWave) {
        const double* wa = W + (16 * rb + m) * g.P + kq;
        const double* xb = X + m * g.KP16 + kq;
        f64x4 acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = zero4<f64x4>();
        for (int k0 = 0; k0 < g.KP16; k0 += 4) {
            const double a = wa[k0];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                if (cb < nt && k0 < 16 * cb + 16)
                    acc[cb] = Mma<double>::step(a, xb[16 * cb * g.KP16 + k0], acc[cb]);
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            if (cb < nt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * rb + Mma<double>::row(kq, r), col = 16 * cb + m;
                    W[row * g.P + col] = acc[cb][r];
                }
            }
        }
    }
}

__host__ __device__ inline CqrGeom cqr_geom(int I, int K) {
    CqrGeom g;
    g.I = I;
    g.K = K;
    g.I16 = (I + 15) & ~15;
    g.KP16 = (K + 15) & ~15;
    g.P = g.KP16 + 1;
    return g;
}

__host__ __device__ inline size_t cqr_w_doubles(const CqrGeom& g) {
    return (static_cast<size_t>(g.I16) * g.P + 1) & ~static_cast<size_t>(1);
}

template <int KB>
__global__ __launch_bounds__(kBlock) void k_cqr(const double* __restrict__ y, int I, int K,
                                                double* work, double* q64, void* q_out, int dbl,
                                                uint32_t* flags) {
    extern __shared__ __align__(16) double shd[];
    const CqrGeom g = cqr_geom(I, K);
    double* W = shd;
    double* G = W + cqr_w_doubles(g);      // Gram, then the broadcast columns / rows of L
    double* X = G + g.KP16 * g.KP16;
    __shared__ double diag0[RHOSVD_MAX_K];
    __shared__ double tau_s[RHOSVD_MAX_K], alpha_s[RHOSVD_MAX_K];
    __shared__ double red[kBlock / kWave];
    __shared__ int ok_sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    // zero padding of W and all of X, then Y (coalesced over i)
    for (int i = wave; i < g.I16; i += kBlock / kWave)
        for (int k = lane; k < g.P; k += kWave)
            if (i >= I || k >= K) W[i * g.P + k] = 0.0;
    for (int e = tid; e < g.KP16 * g.KP16; e += kBlock) X[e] = 0.0;
    {
        const int n = I * K;
        for (int e0 = tid; e0 < n; e0 += 8 * kBlock) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * kBlock;
                v[u] = y[e < n ? e : n - 1];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * kBlock;
                if (e < n) {
                    const int k = e / I, i = e - k * I;
                    W[i * g.P + k] = v[u];
                }
            }
        }
    }
    __syncthreads();
    // One call site for the unrolled factorisation: pass r forms the Gram of
    // the current W, factors it and applies X.  A failed first factorisation
    // restarts with the shift of Fukaya et al. (SISC 2020), s = 11 (I K +
    // K (K + 1)) u ||Y||_F^2 with ||Y||_F^2 = trace(G), and three passes.
    bool shifted = false, ok = true;
    int rounds = 2;
    double shift = 0.0;
    for (int r = 0; r < rounds; ++r) {
        mfma_gram(W, g, G, shift, diag0);
        __syncthreads();
        if (wave == 0) {
            const bool okw = wave_chol_inv<KB>(G, diag0, G, X, K, g.KP16);
            if (tid == 0) ok_sh = okw;
        }
        __syncthreads();
        if (!ok_sh) {
            if (r == 0 && !shifted) {
                double trace = 0.0;
                for (int j = 0; j < K; ++j) trace += diag0[j];
                shift = 11.0 * (static_cast<double>(I) * K + static_cast<double>(K) * (K + 1)) *
                        1.1102230246251565e-16 * trace;
                shifted = true;
                rounds = 3;
                r = -1;
                __syncthreads();
                continue;
            }
            ok = false;
            break;
        }
        shift = 0.0;
        mfma_apply(W, g, X);
        __syncthreads();
    }
    if (ok) {
        for (int e = tid; e < I * K; e += kBlock) {
            const int k = e / I, i = e - k * I;
            const double v = W[i * g.P + k];
            q64[e] = v;
            if (dbl)
                static_cast<double*>(q_out)[e] = v;
            else
                static_cast<float*>(q_out)[e] = static_cast<float>(v);
        }
    } else {
        householder_qr(y, I, K, work, q64, tau_s, alpha_s, red);
        for (int e = tid; e < I * K; e += kBlock) {
            if (dbl)
                static_cast<double*>(q_out)[e] = q64[e];
            else
                static_cast<float*>(q_out)[e] = static_cast<float>(q64[e]);
        }
    }
    if (tid == 0 && flags) {
        uint32_t f = shifted ? RHOSVD_FLAG_CQR_SHIFTED : 0u;
        if (!ok) f |= RHOSVD_FLAG_QR_HOUSEHOLDER;
        if (f) atomicOr(flags, f);
    }
}

static int cqr_kb(int K) { return (K + 7) & ~7; }

size_t cqr_lds_bytes(int64_t I, int K) {
    const CqrGeom g = cqr_geom(static_cast<int>(I), K);
    return (cqr_w_doubles(g) + 2 * static_cast<size_t>(g.KP16) * g.KP16) * sizeof(double);
}

hipError_t launch_reduce_y(bool dbl, const void* part, int G, int I, int K, int I_pad, int K_pad,
                           double* y, hipStream_t s) {
    return launch_reduce_parts(dbl, part, G, I, K, I_pad, K_pad, y, s);
}

hipError_t launch_gram_reduce(bool dbl, const void* part, int G, int K, int K_pad, double* c,
                              hipStream_t s) {
    return launch_reduce_parts(dbl, part, G, K, K, K_pad, K_pad, c, s);
}

hipError_t launch_cqr(const double* y, int64_t I, int K, bool dbl, void* q_out, double* q64,
                      uint32_t* flags, hipStream_t s) {
    if (K > 64 || I > (1 << 20) || cqr_lds_bytes(I, K) + kStaticLdsMargin > kLdsLimit)
        return launch_cqr_global(y, I, K, dbl, q_out, q64, flags, s);
    return launch_cqr_lds(y, I, K, dbl, q_out, q64, flags, s);
}

hipError_t launch_cqr_lds(const double* y, int64_t I, int K, bool dbl, void* q_out, double* q64,
                          uint32_t* flags, hipStream_t s) {
    if (K < 1 || K > 64 || I < 1 || I > (1 << 20)) return hipErrorInvalidValue;
    double* work = q64 + I * K;
    const size_t lds = cqr_lds_bytes(I, K);
    if (lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
    const int Ii = static_cast<int>(I), d = dbl ? 1 : 0;
#define RH_CQR_CASE(KBV)                                                                   \
    case KBV:                                                                              \
        hipLaunchKernelGGL(k_cqr<KBV>, dim3(1), dim3(kBlock), lds, s, y, Ii, K, work, q64, \
                           q_out, d, flags);                                               \
        break;
    switch (cqr_kb(K)) {
        RH_CQR_CASE(8)
        RH_CQR_CASE(16)
        RH_CQR_CASE(24)
        RH_CQR_CASE(32)
        RH_CQR_CASE(40)
        RH_CQR_CASE(48)
        RH_CQR_CASE(56)
        RH_CQR_CASE(64)
        default:
            return hipErrorInvalidValue;
    }
#undef RH_CQR_CASE
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Jacobi EVD (cyclic, round-robin parallel ordering, rotations as in Golub &
// Van Loan sym.schur2) of A (LDS, row-major Ke x Ke, Ke even <= 64) with V
// accumulated.  Round `round` pairs index 0 with one of the others and
// rotates the rest, so that every pair meets once per sweep; the pairs of all
// rounds are tabulated once.  A round: wave 0 computes the Ke/2 rotations
// (c, s, t), then every 2 x 2 block {p1,q1} x {p2,q2} of A (upper block
// triangle, mirrored) becomes J1^T A J2 and every 2 x 2 block of V becomes
// V J2, in place: the blocks partition both matrices.  A thread keeps the
// same blocks (by pair number) for the whole iteration and gathers all its
// operands before it stores anything.  Diagonal blocks take the closed form
// a_pp - t a_pq, a_qq + t a_pq and an exact zero.  Stops when the
// off-diagonal mass is at most 1e-28 of the total (relative RMS 1e-14);
// rotations with a_pq^2 <= 1e-36 |a_pp a_qq| are skipped, and so are rounds
// without a rotation.  A is double-buffered across rounds (see jacobi_lds).
// ---------------------------------------------------------------------------
constexpr int kSweeps = 30;

__device__ __forceinline__ void rr_pair(int m, int round, int Ke, int& p, int& q) {
    const int n1 = Ke - 1;
    int x0 = m - 1 + round;
    if (x0 >= n1) x0 -= n1;
    int x1 = Ke - 2 - m + round;
    if (x1 >= n1) x1 -= n1;
    const int a0 = (m == 0) ? 0 : 1 + x0;
    const int a1 = 1 + x1;
    p = a0 < a1 ? a0 : a1;
    q = a0 < a1 ? a1 : a0;
}

// 1 / x and 1 / sqrt(x) from the hardware estimates with one Newton step.
__device__ __forceinline__ double rcp_nr(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return fma(fma(-x, y, 1.0), y, y);
}
__device__ __forceinline__ double rsq_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double r = fma(-x * y, y, 1.0);
    return fma(0.5 * y, r, y);
}

// Rotation (c, s, t) annihilating a_pq (Golub & Van Loan sym.schur2):
// tau = (a_qq - a_pp) / (2 a_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
// c = 1 / sqrt(1 + t^2), s = t c; evaluated as t = sign(d) e / (|d| +
// sqrt(d^2 + e^2)) with d = a_qq - a_pp, e = 2 a_pq scaled by a power of two.
__device__ __forceinline__ void sym_schur2(double app, double aqq, double apq, double& c,
                                           double& s, double& t) {
    const double d = aqq - app, e = 2.0 * apq;
    const int ed = __builtin_amdgcn_frexp_exp(d), ee = __builtin_amdgcn_frexp_exp(e);
    const int ex = ed > ee ? ed : ee;
    const double dn = __builtin_amdgcn_ldexp(d, -ex), en = __builtin_amdgcn_ldexp(e, -ex);
    const double h = fma(dn, dn, en * en);
    const double r = h * rsq_nr(h);
    t = (d >= 0.0 ? en : -en) * rcp_nr(fabs(dn) + r);
    c = rsq_nr(fma(t, t, 1.0));
    s = t * c;
}

constexpr int kJacItems = 7;   // (Ke/2)(Ke/2 + 1)/2 + (Ke/2)^2 <= 7 * 256 for Ke <= 64

// pq: (Ke - 1) x (Ke / 2) table of pairs, p | q << 8.  One workgroup
// barrier per round: every wave computes all of the round's rotations itself
// (lanes < Ke/2, into its own LDS slot), A is read from one buffer and
// written to the other (A2), and V, whose blocks only their owner touches
// within a round, is updated in place.  All waves see the same A and take the
// same decisions (round skips, convergence).  On return A points at the
// current buffer.
__device__ bool jacobi_lds(double*& A, double* A2, double* V, int Ke, unsigned short* pq,
                           int* sweeps) {
    __shared__ double rot[kBlock / kWave][3][RHOSVD_MAX_K / 2];
    __shared__ double red[2][kBlock / kWave];
    __shared__ int conv;
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    const int half = Ke / 2;
    const int n1 = Ke - 1;
    const int nA = half * (half + 1) / 2;   // A blocks (m1 <= m2)
    const int nV = half * half;             // V blocks (row pair, column pair)
    double* const A0 = A;                   // the two buffers: the initial A and A2
    double* rc = rot[wave][0];
    double* rs = rot[wave][1];
    double* rt = rot[wave][2];
    for (int e = tid; e < n1 * half; e += kBlock) {
        const int round = e / half, m = e - round * half;
        int p, q;
        rr_pair(m, round, Ke, p, q);
        pq[e] = static_cast<unsigned short>(p | (q << 8));
    }
    // this thread's items for the whole iteration: A block (m1 <= m2) or V
    // block (row pair m1 - 64, column pair m2); m1 < 0 marks no item
    int item_m1[kJacItems], item_m2[kJacItems];
#pragma unroll
    for (int u = 0; u < kJacItems; ++u) {
        const int it = tid + u * kBlock;
        int m1 = -1, m2 = 0;
        if (it < nA) {
            int rem = it;
            m1 = 0;
            while (rem >= half - m1) {
                rem -= half - m1;
                ++m1;
            }
            m2 = m1 + rem;
        } else if (it < nA + nV) {
            const int v = it - nA;
            m1 = 64 + v / half;
            m2 = v % half;
        }
        item_m1[u] = m1;
        item_m2[u] = m2;
    }
    __syncthreads();
    for (int sweep = 0; sweep < kSweeps; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < Ke * Ke; e += kBlock) {
            const int r = e / Ke, c = e - r * Ke;
            const double v = A[e] * A[e];
            tot += v;
            if (r != c) off += v;
        }
        off = wave_sum(off);
        tot = wave_sum(tot);
        if (lane == 0) {
            red[0][wave] = off;
            red[1][wave] = tot;
        }
        __syncthreads();
        if (tid == 0) {
            double o = 0.0, t = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w) {
                o += red[0][w];
                t += red[1][w];
            }
            conv = (o <= 1e-28 * t) ? 1 : 0;
        }
        __syncthreads();
        *sweeps = sweep;
        if (conv) return true;
        for (int round = 0; round < n1; ++round) {
            const unsigned short* pr = pq + round * half;
            // the pairs of this thread's blocks (the table is read-only)
            int code1[kJacItems], code2[kJacItems];
#pragma unroll
            for (int u = 0; u < kJacItems; ++u) {
                const int m1 = item_m1[u], m2 = item_m2[u];
                code1[u] = (m1 >= 0 && m1 < 64) ? pr[m1] : 0;
                code2[u] = (m1 >= 0) ? pr[m2] : 0;
            }
            int rotate = 0;
            if (lane < half) {
                const int code = pr[lane];
                const int p = code & 0xff, q = code >> 8;
                const double apq = A[p * Ke + q];
                const double app = A[p * Ke + p], aqq = A[q * Ke + q];
                double c = 1.0, sn = 0.0, t = 0.0;
                if (apq * apq > 1e-36 * fabs(app * aqq)) {
                    sym_schur2(app, aqq, apq, c, sn, t);
                    rotate = 1;
                }
                rc[lane] = c;
                rs[lane] = sn;
                rt[lane] = t;
            }
            if (__ballot(rotate) == 0ull) continue;   // same in every wave
            double* An = (A == A0) ? A2 : A0;
            double x[kJacItems][4], cs[kJacItems][4];
#pragma unroll
            for (int u = 0; u < kJacItems; ++u) {
                const int m1 = item_m1[u], m2 = item_m2[u];
                if (m1 < 0) continue;
                const int p2 = code2[u] & 0xff, q2 = code2[u] >> 8;
                cs[u][2] = rc[m2];
                cs[u][3] = rs[m2];
                if (m1 < 64) {
                    const int p1 = code1[u] & 0xff, q1 = code1[u] >> 8;
                    cs[u][0] = (m1 == m2) ? rt[m1] : rc[m1];
                    cs[u][1] = rs[m1];
                    x[u][0] = A[p1 * Ke + p2];
                    x[u][1] = A[p1 * Ke + q2];
                    x[u][2] = A[q1 * Ke + p2];
                    x[u][3] = A[q1 * Ke + q2];
                } else {
                    const int i0 = 2 * (m1 - 64);
                    x[u][0] = V[i0 * Ke + p2];
                    x[u][1] = V[i0 * Ke + q2];
                    x[u][2] = V[(i0 + 1) * Ke + p2];
                    x[u][3] = V[(i0 + 1) * Ke + q2];
                }
            }
#pragma unroll
            for (int u = 0; u < kJacItems; ++u) {
                const int m1 = item_m1[u], m2 = item_m2[u];
                if (m1 < 0) continue;
                const int p2 = code2[u] & 0xff, q2 = code2[u] >> 8;
                const double c2 = cs[u][2], s2 = cs[u][3];
                if (m1 >= 64) {
                    const int i0 = 2 * (m1 - 64);
                    V[i0 * Ke + p2] = c2 * x[u][0] - s2 * x[u][1];
                    V[i0 * Ke + q2] = s2 * x[u][0] + c2 * x[u][1];
                    V[(i0 + 1) * Ke + p2] = c2 * x[u][2] - s2 * x[u][3];
                    V[(i0 + 1) * Ke + q2] = s2 * x[u][2] + c2 * x[u][3];
                } else if (m1 == m2) {
                    const double t = cs[u][0];
                    const double apq = x[u][1];
                    An[p2 * Ke + p2] = x[u][0] - t * apq;
                    An[q2 * Ke + q2] = x[u][3] + t * apq;
                    An[p2 * Ke + q2] = 0.0;
                    An[q2 * Ke + p2] = 0.0;
                } else {
                    const int p1 = code1[u] & 0xff, q1 = code1[u] >> 8;
                    const double c1 = cs[u][0], s1 = cs[u][1];
                    const double a = x[u][0], b = x[u][1], d = x[u][2], e = x[u][3];
                    const double t00 = c2 * a - s2 * b, t01 = s2 * a + c2 * b;
                    const double t10 = c2 * d - s2 * e, t11 = s2 * d + c2 * e;
                    const double n00 = c1 * t00 - s1 * t10, n01 = c1 * t01 - s1 * t11;
                    const double n10 = s1 * t00 + c1 * t10, n11 = s1 * t01 + c1 * t11;
                    An[p1 * Ke + p2] = n00;
                    An[p1 * Ke + q2] = n01;
                    An[q1 * Ke + p2] = n10;
                    An[q1 * Ke + q2] = n11;
                    An[p2 * Ke + p1] = n00;
                    An[q2 * Ke + p1] = n01;
                    An[p2 * Ke + q1] = n10;
                    An[q2 * Ke + q1] = n11;
                }
            }
            __syncthreads();
            A = An;
        }
    }
    return false;
}

// EVD of C (K x K, column-major, device) and, when q != nullptr, the factor
// step: U = Q V[:, :R] (V = identity when use_v == 0), canonical signs,
// M = V_R diag(s) (K x R), sigma = sqrt(max(lambda, 0))[:R].  Q is staged
// into LDS (row-major, pitch K16 = 16 ceil(K / 16), zero-padded to I16 rows)
// together with C, so its load overlaps nothing but C's; U is formed on the
// f64 matrix cores in place of Q, one 16-row block per wave at a time.  The
// sorted eigenpairs also go to v_out / lam_out when those are non-null.
template <typename T, bool STAGED>
__global__ __launch_bounds__(kBlock) void k_evd_factor(const double* __restrict__ cin, int K,
                                                       double* v_out, double* lam_out,
                                                       uint32_t* flags, const T* __restrict__ q,
                                                       int I, int R, int use_v,
                                                       T* __restrict__ u_out,
                                                       T* __restrict__ m_out,
                                                       double* __restrict__ sigma,
                                                       double* __restrict__ qwork) {
    extern __shared__ __align__(16) double shd[];
    const int Ke = K + (K & 1);
    const int K16 = (K + 15) & ~15, I16 = (I + 15) & ~15;
    double* A = shd;
    double* A2 = A + Ke * Ke;
    double* V = A2 + Ke * Ke;
    // Q staged as I16 x K16 (row-major): in LDS when it fits, else in qwork
    double* Qs = STAGED ? V + Ke * Ke : qwork;
    unsigned short* pq = reinterpret_cast<unsigned short*>(V + Ke * Ke + (STAGED && q ? I16 * K16 : 0));
    __shared__ double lam[RHOSVD_MAX_K], dg[RHOSVD_MAX_K];
    __shared__ double sgn[RHOSVD_MAX_K];
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    for (int e = tid; e < Ke * Ke; e += kBlock) {
        const int r = e / Ke, c = e - r * Ke;
        A[e] = (r < K && c < K) ? cin[c * K + r] : 0.0;
        V[e] = (r == c) ? 1.0 : 0.0;
    }
    if (q) {
        for (int e = tid; e < I16 * K16; e += kBlock) {
            // (a row of Q per K16 consecutive entries)
            const int i = e / K16, k = e - i * K16;
            Qs[e] = (i < I && k < K) ? static_cast<double>(q[static_cast<int64_t>(k) * I + i]) : 0.0;
        }
    }
    __syncthreads();
    int sweeps = 0;
    const bool conv = jacobi_lds(A, A2, V, Ke, pq, &sweeps);
    if (tid == 0 && !conv && flags) atomicOr(flags, RHOSVD_FLAG_EVD_NOCONV);
    // the stand-alone EVD reports its sweep count in bits 16..23 of flags
    if (tid == 0 && flags && !q) atomicOr(flags, static_cast<uint32_t>(sweeps & 0xff) << 16);
    for (int i = tid; i < K; i += kBlock) dg[i] = A[i * Ke + i];
    __syncthreads();
    double* Vs = (A == shd) ? A2 : shd;   // sorted eigenvectors (K x K, column-major), free buffer
    for (int i = tid; i < K; i += kBlock) {
        const double li = dg[i];
        int rank = 0;
        for (int j = 0; j < K; ++j) {
            const double lj = dg[j];
            rank += (lj > li) || (lj == li && j < i);
        }
        lam[rank] = li;
        for (int k = 0; k < K; ++k) Vs[rank * K + k] = V[k * Ke + i];
    }
    __syncthreads();
    if (v_out)
        for (int e = tid; e < K * K; e += kBlock) v_out[e] = Vs[e];
    if (lam_out)
        for (int e = tid; e < K; e += kBlock) lam_out[e] = lam[e];
    if (!q) return;
    // U = Q V_R (FP64), 16 x 16 tiles, written over Q's rows (pitch K16 >= R)
    {
        const int m = lane & 15, kq = lane >> 4;
        const int nib = I16 >> 4, nrb = (R + 15) >> 4;
        for (int ib = wave; ib < nib; ib += kBlock / kWave) {
            const double* qa = Qs + (16 * ib + m) * K16 + kq;
            f64x4 acc[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) acc[rb] = zero4<f64x4>();
            for (int k0 = 0; k0 < K16; k0 += 4) {
                const double a = qa[k0];
                const int k = k0 + kq;
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    if (rb < nrb) {
                        const int rcol = 16 * rb + m;
                        double b = 0.0;
                        if (rcol < R && k < K) b = use_v ? Vs[rcol * K + k] : (k == rcol ? 1.0 : 0.0);
                        acc[rb] = Mma<double>::step(a, b, acc[rb]);
                    }
                }
            }
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                if (rb < nrb) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * ib + Mma<double>::row(kq, r), col = 16 * rb + m;
                        if (col < R) Qs[row * K16 + col] = acc[rb][r];
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int r = wave; r < R; r += kBlock / kWave) {
        double best = -1.0;
        int bi = 0x7fffffff;
        for (int i = lane; i < I; i += kWave) {
            const double a = fabs(Qs[i * K16 + r]);
            if (a > best) {
                best = a;
                bi = i;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, kWave);
            const int oi = __shfl_xor(bi, o, kWave);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (lane == 0) sgn[r] = (Qs[bi * K16 + r] < 0.0) ? -1.0 : 1.0;
    }
    __syncthreads();
    for (int e = tid; e < I * R; e += kBlock) {
        const int r = e / I, i = e - r * I;
        u_out[e] = static_cast<T>(sgn[r] * Qs[i * K16 + r]);
    }
    for (int e = tid; e < K * R; e += kBlock) {
        const int r = e / K, k = e - r * K;
        const double vv = use_v ? Vs[r * K + k] : (k == r ? 1.0 : 0.0);
        m_out[e] = static_cast<T>(sgn[r] * vv);
    }
    if (sigma)
        for (int r = tid; r < R; r += kBlock) sigma[r] = sqrt(fmax(lam[r], 0.0));
}

// LDS of k_evd_factor: A, A2 and V (Ke x Ke each), Q staged as I16 x K16 when
// the factor step runs and it fits, and the (Ke - 1) x (Ke / 2) pair table.
size_t evd_lds_bytes(int K, int64_t I, bool staged) {
    const int Ke = K + (K & 1);
    const size_t K16 = (K + 15) & ~15, I16 = (I + 15) & ~static_cast<int64_t>(15);
    size_t b = 3 * static_cast<size_t>(Ke) * Ke * sizeof(double);
    if (staged) b += I16 * K16 * sizeof(double);
    b += static_cast<size_t>(Ke - 1) * (Ke / 2) * sizeof(unsigned short);
    return (b + 15) & ~static_cast<size_t>(15);
}

size_t evd_qwork_doubles(int K, int64_t I) {
    return static_cast<size_t>((I + 15) & ~static_cast<int64_t>(15)) * ((K + 15) & ~15);
}

// u64: I16 x K16 doubles of device scratch, used when Q does not fit in LDS.
hipError_t launch_evd_factor(bool dbl, const double* c, int K, double* v_out, double* lam_out,
                             uint32_t* flags, const void* q, int64_t I, int R, int use_v,
                             void* u_out, void* m_out, double* sigma, double* u64, hipStream_t s) {
    if (K < 1 || K > 64) return hipErrorInvalidValue;
    if (q && (I < 1 || I > (1 << 24) || R < 1 || R > K)) return hipErrorInvalidValue;
    const bool staged = q != nullptr && evd_lds_bytes(K, I, true) + kStaticLdsMargin <= kLdsLimit;
    if (q && !staged && !u64) return hipErrorInvalidValue;
    const size_t lds = evd_lds_bytes(K, I, staged);
    if (lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
    const int Ii = static_cast<int>(I);
#define RH_EVD_LAUNCH(T, ST)                                                                      \
    hipLaunchKernelGGL((k_evd_factor<T, ST>), dim3(1), dim3(kBlock), lds, s, c, K, v_out, lam_out, \
                       flags, static_cast<const T*>(q), Ii, R, use_v, static_cast<T*>(u_out),     \
                       static_cast<T*>(m_out), sigma, u64)
    if (dbl) {
        if (staged) RH_EVD_LAUNCH(double, true); else RH_EVD_LAUNCH(double, false);
    } else {
        if (staged) RH_EVD_LAUNCH(float, true); else RH_EVD_LAUNCH(float, false);
    }
#undef RH_EVD_LAUNCH
    return hipGetLastError();
}

hipError_t launch_evd(const double* c, int K, double* v, double* lambda, uint32_t* flags,
                      hipStream_t s) {
    return launch_evd_factor(true, c, K, v, lambda, flags, nullptr, 0, 0, 0, nullptr, nullptr,
                             nullptr, nullptr, s);
}

}  // namespace rh
