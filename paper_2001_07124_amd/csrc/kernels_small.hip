// Small dense steps between the streaming passes, written for latency:
//   k_reduce_parts  fixed-order sum of per-workgroup partials (many workgroups)
//   k_cqr           CholeskyQR2 of Y (I x K) with Y resident in LDS: Gram and
//                   triangular update on the f64 matrix cores, the K x K
//                   Cholesky factor and its inverse in one wave's registers
//                   (Algorithm 1 step 3)
//   k_hqr           Householder QR of Y in one workgroup (step 3)
//   k_evd_tri       symmetric EVD of the K x K Gram (Algorithm 1 step 5) by
//                   tridiagonalisation, multisection and inverse iteration,
//                   fused with U = Q V[:, :R], sign canonicalisation, M = V_R
//                   and sigma (steps 6-7)
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "device_common.hpp"
#include "householder.hpp"
#include "kernels.hpp"
#include "rhosvd.h"

namespace rh {

// ---------------------------------------------------------------------------
// out[e] = sum_g part[g * stride + off(e)], e < I K, in a fixed order.
// Block: 16 elements x 16 partial groups; group q sums g = q, q + 16, ...
// eight loads at a time, and the groups are added in order through LDS.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void reduce_parts_body(const T* __restrict__ part, int G, int I, int K,
                                                  int I_pad, int K_pad, double* __restrict__ y,
                                                  int blk) {
    constexpr int kE = 16, kG = kBlock / kE;
    __shared__ double red[kG][kE + 1];
    const int el = threadIdx.x % kE, q = threadIdx.x / kE;
    const int e = blk * kE + el;
    double s = 0.0;
    if (e < I * K) {
        const int k = e / I, i = e - k * I;
        const size_t stride = static_cast<size_t>(K_pad) * I_pad;
        const T* p = part + static_cast<size_t>(k) * I_pad + i;
        int g = q;
        for (; g + 7 * kG < G; g += 8 * kG) {
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = static_cast<double>(p[(g + u * kG) * stride]);
            s += ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        }
        for (; g < G; g += kG) s += static_cast<double>(p[g * stride]);
    }
    red[q][el] = s;
    __syncthreads();
    if (q == 0 && e < I * K) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < kG; ++j) t += red[j][el];
        y[e] = t;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_reduce_parts(const T* __restrict__ part, int G, int I,
                                                         int K, int I_pad, int K_pad,
                                                         double* __restrict__ y) {
    reduce_parts_body<T>(part, G, I, K, I_pad, K_pad, y, blockIdx.x);
}

// Batch: the items' passes have few partials (at most the workgroups per
// item), so each thread sums one element's G partials itself, in ascending
// order with eight loads in flight; workgroup (x, y) takes elements
// 256 x .. 256 x + 255 of job y (blocks past the job's I K return).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_reduce_parts_batch(const ReduceJob* __restrict__ jobs) {
    const ReduceJob& j = jobs[blockIdx.y];
    const int e = static_cast<int>(blockIdx.x) * kBlock + static_cast<int>(threadIdx.x);
    if (e >= j.I * j.K) return;
    const int k = e / j.I, i = e - k * j.I;
    const size_t stride = static_cast<size_t>(j.K_pad) * j.I_pad;
    const T* __restrict__ p = static_cast<const T*>(j.part) + static_cast<size_t>(k) * j.I_pad + i;
    double sum = 0.0;
    int g = 0;
    for (; g + 8 <= j.G; g += 8) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = static_cast<double>(p[(g + u) * stride]);
#pragma unroll
        for (int u = 0; u < 8; ++u) sum += a[u];
    }
    for (; g < j.G; ++g) sum += static_cast<double>(p[g * stride]);
    j.y[e] = sum;
}

hipError_t launch_reduce_parts_batch(bool dbl, const ReduceJob* jobs, int njobs, int max_elems,
                                     hipStream_t s) {
    if (njobs < 1 || max_elems < 1) return hipErrorInvalidValue;
    const dim3 grid((max_elems + kBlock - 1) / kBlock, njobs);
    if (dbl)
        hipLaunchKernelGGL(k_reduce_parts_batch<double>, grid, dim3(kBlock), 0, s, jobs);
    else
        hipLaunchKernelGGL(k_reduce_parts_batch<float>, grid, dim3(kBlock), 0, s, jobs);
    return hipGetLastError();
}

hipError_t launch_reduce_parts(bool dbl, const void* part, int G, int I, int K, int I_pad,
                               int K_pad, double* y, hipStream_t s) {
    const dim3 grid((I * K + 15) / 16);
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
    int GP;   // pitch of G and X (KP16 + 1: odd, so a column walk spreads over the banks)
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
                G[row * g.GP + col] = x;
                G[col * g.GP + row] = x;
                if (row == col) diag0[row] = x;
            }
        }
    }
}

// The same Gram for NT = KP16 / 16 >= 3 column tiles, split by rows: wave w
// takes the rows [w I16 / 4, (w + 1) I16 / 4) and forms all NT (NT + 1) / 2
// upper tiles, each k-step loading its NT fragments once.  Waves 1..3 leave
// their tiles in red (3 NP 256 doubles: the G and X region, which holds
// 2 KP16 (KP16 + 1) >= 3 NP 256 for NT >= 3); wave 0 adds them in wave order and
// writes G.  X must be rewritten (zero padding included) before its next use.
template <int NT>
__device__ void mfma_gram_rows(const double* W, const CqrGeom g, double* G, double* red,
                               double shift, double* diag0) {
    constexpr int NP = NT * (NT + 1) / 2;
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int m = lane & 15, kq = lane >> 4;
    const int rows = g.I16 >> 2;
    const double* wp = W + (wave * rows + kq) * g.P + m;
    f64x4 acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = zero4<f64x4>();
#pragma unroll 4
    for (int i0 = 0; i0 < rows; i0 += 4) {
        double a[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) a[t] = wp[i0 * g.P + 16 * t];
        int p = 0;
#pragma unroll
        for (int ta = 0; ta < NT; ++ta)
#pragma unroll
            for (int tb = ta; tb < NT; ++tb) {
                acc[p] = Mma<double>::step(a[ta], a[tb], acc[p]);
                ++p;
            }
    }
    if (wave > 0) {
        double* rw = red + static_cast<size_t>(wave - 1) * NP * 256 + lane * 4;
#pragma unroll
        for (int p = 0; p < NP; ++p) *reinterpret_cast<f64x4*>(rw + p * 256) = acc[p];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const f64x4 o = *reinterpret_cast<const f64x4*>(red + (w * NP + p) * 256 + lane * 4);
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[p][r] += o[r];
            }
        int p = 0;
#pragma unroll
        for (int ta = 0; ta < NT; ++ta)
#pragma unroll
            for (int tb = ta; tb < NT; ++tb) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * ta + Mma<double>::row(kq, r), col = 16 * tb + m;
                    if (row < g.K && col < g.K) {
                        const double x = acc[p][r] + (row == col ? shift : 0.0);
                        G[row * g.GP + col] = x;
                        G[col * g.GP + row] = x;
                        if (row == col) diag0[row] = x;
                    }
                }
                ++p;
            }
    }
}

// One wave.  Right-looking Cholesky G = L L^T with lane i holding row i:
// step j takes the pivot from lane j, L(j+1, j) by a lane read (the next
// pivot depends on nothing else), and the rest of column j through S.  Then
// X = L^{-1} by rows, lane i solving x L = e_i from the last column down with
// the rows of L broadcast from S.  S may alias G (read into registers first);
// it must be 16-byte aligned and hold K rows of pitch SP = XP rounded up to
// even (the broadcast rows are read two doubles per instruction), which may
// run into X: X is written last.  Out: X (pitch XP; rows >= K zero).  Returns
// false, uniformly, on a pivot not above 1e-14 of its original diagonal.
template <int KB>
__device__ bool wave_chol_inv(const double* G, const double* diag0, double* S, double* X, int K,
                              int XP, int XN) {
    const int lane = threadIdx.x & 63;
    const int li = lane < KB ? lane : KB - 1;
    double g[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) g[c] = (li < K && c < K) ? G[li * XP + c] : (li == c ? 1.0 : 0.0);
    const double dgl = (li < K) ? diag0[li] : 1.0;
    const int SP = (XP + 1) & ~1;
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
                    if (lane < KB) S[j * SP + lane] = l;
                    double sr[KB];
#pragma unroll
                    for (int c = (j + 2) & ~1; c < KB; c += 2) {
                        const double2 v = *reinterpret_cast<const double2*>(S + j * SP + c);
                        sr[c] = v.x;
                        sr[c + 1] = v.y;
                    }
#pragma unroll
                    for (int c = j + 2; c < KB; ++c) g[c] = fma(-l, sr[c], g[c]);
                }
            }
        }
    }
    if (!ok) return false;
    if (lane < KB) {
#pragma unroll
        for (int c = 0; c < KB; ++c) S[lane * SP + c] = g[c];
    }
    double acc[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) acc[k] = 0.0;
#pragma unroll
    for (int m = KB - 1; m >= 0; --m) {
        if (m < K) {
            double sr[KB];
#pragma unroll
            for (int k = 0; k < m; k += 2) {
                const double2 v = *reinterpret_cast<const double2*>(S + m * SP + k);
                sr[k] = v.x;
                sr[k + 1] = v.y;
            }
            const double x = ((li == m ? 1.0 : 0.0) - acc[m]) * readlane_d(dinvl, m);
            acc[m] = x;
#pragma unroll
            for (int k = 0; k < m; ++k) acc[k] = fma(x, sr[k], acc[k]);
        } else {
            acc[m] = 0.0;
        }
    }
    // all of X's XN x XN block (pitch XP): zero outside K x K
    for (int r = lane; r < XN; r += kWave) {
        const bool in = r < K;
#pragma unroll
        for (int c = 0; c < KB; ++c) X[r * XP + c] = in ? acc[c] : 0.0;
        for (int c = KB; c < XN; ++c) X[r * XP + c] = 0.0;
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
        const double* xb = X + m * g.GP + kq;
        f64x4 acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = zero4<f64x4>();
        for (int k0 = 0; k0 < g.KP16; k0 += 4) {
            const double a = wa[k0];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                if (cb < nt && k0 < 16 * cb + 16)
                    acc[cb] = Mma<double>::step(a, xb[16 * cb * g.GP + k0], acc[cb]);
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

// W <- W X^T as mfma_apply, with X's fragments (lower triangular: column tile
// cb needs k < 16 cb + 16) held in registers across the row blocks and each
// block's W fragments loaded at once.
template <int NT>
__device__ void mfma_apply_rows(double* W, const CqrGeom g, const double* X) {
    constexpr int NK = 4 * NT;   // k-steps of 4 over KP16
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int m = lane & 15, kq = lane >> 4;
    double xb[NT][NK];
#pragma unroll
    for (int cb = 0; cb < NT; ++cb)
#pragma unroll
        for (int st = 0; st < NK; ++st)
            xb[cb][st] = (st < 4 * cb + 4) ? X[(16 * cb + m) * g.GP + 4 * st + kq] : 0.0;
    const int nrb = g.I16 >> 4;
    for (int rb = wave; rb < nrb; rb += kBlock / kWave) {
        double a[NK];
#pragma unroll
        for (int st = 0; st < NK; ++st) a[st] = W[(16 * rb + m) * g.P + 4 * st + kq];
        f64x4 acc[NT];
#pragma unroll
        for (int cb = 0; cb < NT; ++cb) {
            acc[cb] = zero4<f64x4>();
#pragma unroll
            for (int st = 0; st < 4 * cb + 4; ++st) acc[cb] = Mma<double>::step(a[st], xb[cb][st], acc[cb]);
        }
#pragma unroll
        for (int cb = 0; cb < NT; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * rb + Mma<double>::row(kq, r), col = 16 * cb + m;
                W[row * g.P + col] = acc[cb][r];
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
    g.GP = g.KP16 + 1;
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
    double* X = G + g.KP16 * g.GP;
    __shared__ double diag0[RHOSVD_MAX_K];
    __shared__ double tau_s[RHOSVD_MAX_K], alpha_s[RHOSVD_MAX_K];
    __shared__ double red[kBlock / kWave];
    __shared__ int ok_sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    // zero padding of W (rows I.. as one range, columns K.. one row per
    // thread) and all of X, then Y (coalesced over i)
    {
        const int r0 = I * g.P, r1 = g.I16 * g.P;
        for (int e = r0 + tid; e < r1; e += kBlock) W[e] = 0.0;
        for (int i = tid; i < I; i += kBlock)
            for (int k = K; k < g.P; ++k) W[i * g.P + k] = 0.0;
        for (int e = tid; e < g.KP16 * g.GP; e += kBlock) X[e] = 0.0;
    }
    {
        // element e = k I + i of y; (k, i) advanced by kBlock per step
        const int n = I * K;
        for (int e0 = tid; e0 < n; e0 += 32 * kBlock) {
            double v[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                const int e = e0 + u * kBlock;
                v[u] = y[e < n ? e : n - 1];
            }
            int k = e0 / I, i = e0 - k * I;
            const int dk = kBlock / I, di = kBlock - dk * I;
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                if (e0 + u * kBlock < n) W[i * g.P + k] = v[u];
                i += di;
                k += dk;
                if (i >= I) {
                    i -= I;
                    ++k;
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
    // column tiles: K in (KB - 8, KB] gives KP16 = 16 NT
    constexpr int NT = (KB + 15) / 16;
    for (int r = 0; r < rounds; ++r) {
        if constexpr (NT >= 3)
            mfma_gram_rows<NT>(W, g, G, G, shift, diag0);
        else
            mfma_gram(W, g, G, shift, diag0);
        __syncthreads();
        if (wave == 0) {
            const bool okw = wave_chol_inv<KB>(G, diag0, G, X, K, g.GP, g.KP16);
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
        if constexpr (NT >= 3)
            mfma_apply_rows<NT>(W, g, X);
        else
            mfma_apply(W, g, X);
        __syncthreads();
    }
    if (ok) {
        // element e = k I + i, eight LDS reads in flight per thread
        const int n = I * K;
        const int dk = kBlock / I, di = kBlock - dk * I;
        for (int e0 = tid; e0 < n; e0 += 8 * kBlock) {
            int k = e0 / I, i = e0 - k * I;
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                v[u] = (e0 + u * kBlock < n) ? W[i * g.P + k] : 0.0;
                i += di;
                k += dk;
                if (i >= I) {
                    i -= I;
                    ++k;
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * kBlock;
                if (e < n) {
                    q64[e] = v[u];
                    if (dbl)
                        static_cast<double*>(q_out)[e] = v[u];
                    else
                        static_cast<float*>(q_out)[e] = static_cast<float>(v[u]);
                }
            }
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
    return (cqr_w_doubles(g) + 2 * static_cast<size_t>(g.KP16) * g.GP) * sizeof(double);
}

hipError_t launch_reduce_y(bool dbl, const void* part, int G, int I, int K, int I_pad, int K_pad,
                           double* y, hipStream_t s) {
    return launch_reduce_parts(dbl, part, G, I, K, I_pad, K_pad, y, s);
}

hipError_t launch_gram_reduce(bool dbl, const void* part, int G, int K, int K_pad, double* c,
                              hipStream_t s) {
    return launch_reduce_parts(dbl, part, G, K, K, K_pad, K_pad, c, s);
}

hipError_t launch_hqr_fwd(const double* y, int I, int K, bool dbl, void* q_out, double* q64,
                          hipStream_t s);

hipError_t launch_cqr(const double* y, int64_t I, int K, bool dbl, void* q_out, double* q64,
                      uint32_t* flags, hipStream_t s) {
    // a mode of up to 256 rows (512 rows for K <= 32): one Householder QR
    // pass (no breakdown, so flags stay untouched); otherwise CholeskyQR2
    if (K >= 1 && I >= K && ((K <= 64 && I <= 256) || (K <= 32 && I <= 512)))
        return launch_hqr_fwd(y, static_cast<int>(I), K, dbl, q_out, q64, s);
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
// Least-squares operator of the single-pass core recovery (R-PET, Algorithm 9;
// the second sketch of eqs. Onepass / Onepass2, Section 3.1): for
// A = Omt^T Q (S x K, Omt: I x S, Q: I x K, both column-major, S >= K),
// P^T = (pinv(A))^T = A (A^T A)^{-1} (S x K column-major), in FP64 from the
// normal equations: A is a Gaussian sketch of an orthonormal basis, so
// cond(A) is a small constant (about (sqrt(S) + sqrt(K)) / (sqrt(S) - sqrt(K))
// for S = 2K + 1) and squaring it costs nothing.  One workgroup:
//   A = Omt^T Q                 all threads, fixed-order sums over I
//   G = A^T A                   all threads
//   G = L L^T, X = L^{-1}       wave 0 (as CholeskyQR); a breakdown retries
//                               with the shift of Fukaya et al. and sets
//                               RHOSVD_FLAG_CQR_SHIFTED
//   B = A X^T, P^T = B X        one row of A per thread, in place
// LDS: A (S rows of pitch K | 1), then G and X (KP16 rows of pitch KP16 + 1).
// ---------------------------------------------------------------------------
__host__ __device__ inline size_t lsq_lds_doubles(int S, int K) {
    const int KP = K | 1, KP16 = (K + 15) & ~15;
    return static_cast<size_t>(S) * KP + 2 * static_cast<size_t>(KP16) * (KP16 + 1) + 2 * KP16 + 2;
}

template <int KB, typename T>
__global__ __launch_bounds__(kBlock) void k_lsq_pinv(const T* __restrict__ omt,
                                                     const T* __restrict__ q, int I, int S, int K,
                                                     T* __restrict__ pt, uint32_t* flags) {
    extern __shared__ __align__(16) double shd[];
    __shared__ double diag0[RHOSVD_MAX_K];
    __shared__ double shift_sh;
    __shared__ int ok_sh;
    const int KP = K | 1, KP16 = (K + 15) & ~15, GP = KP16 + 1;
    double* A = shd;
    double* G = A + ((static_cast<size_t>(S) * KP + 1) & ~static_cast<size_t>(1));
    double* X = G + static_cast<size_t>(KP16) * GP;
    const int tid = threadIdx.x, wave = wave_id();
    for (int e = tid; e < S * K; e += kBlock) {
        const int r = e / K, k = e - r * K;
        const T* oc = omt + static_cast<size_t>(r) * I;
        const T* qc = q + static_cast<size_t>(k) * I;
        double acc = 0.0;
        for (int i = 0; i < I; ++i) acc = fma(static_cast<double>(oc[i]), static_cast<double>(qc[i]), acc);
        A[r * KP + k] = acc;
    }
    __syncthreads();
    for (int round = 0; round < 2; ++round) {
        for (int e = tid; e < K * K; e += kBlock) {
            const int k1 = e / K, k2 = e - k1 * K;
            double acc = 0.0;
            for (int r = 0; r < S; ++r) acc = fma(A[r * KP + k1], A[r * KP + k2], acc);
            G[k1 * GP + k2] = acc;
            if (k1 == k2) diag0[k1] = acc;
        }
        __syncthreads();
        if (round == 1) {
            // shift s = 11 (S K + K (K + 1)) u trace(G) on the diagonal
            if (tid == 0) {
                double tr = 0.0;
                for (int k = 0; k < K; ++k) tr += diag0[k];
                shift_sh = 11.0 * (static_cast<double>(S) * K + static_cast<double>(K) * (K + 1)) *
                           1.1102230246251565e-16 * tr;
            }
            __syncthreads();
            if (tid < K) {
                G[tid * GP + tid] += shift_sh;
                diag0[tid] += shift_sh;
            }
            __syncthreads();
        }
        if (wave == 0) {
            const bool okw = wave_chol_inv<KB>(G, diag0, G, X, K, GP, KP16);
            if (threadIdx.x == 0) ok_sh = okw;
        }
        __syncthreads();
        if (ok_sh) break;
        if (round == 1) {
            // still singular: Q is rank deficient; report and leave P^T zero
            if (tid == 0 && flags) atomicOr(flags, RHOSVD_FLAG_CQR_SHIFTED | RHOSVD_FLAG_EVD_NOCONV);
            for (int e = tid; e < S * K; e += kBlock) pt[e] = static_cast<T>(0);
            return;
        }
        if (tid == 0 && flags) atomicOr(flags, RHOSVD_FLAG_CQR_SHIFTED);
    }
    // row r of A: B = A X^T (descending k: B(r, k) needs A(r, m <= k)), then
    // P^T = B X (ascending k: needs B(r, m >= k)); X is lower triangular
    for (int r = tid; r < S; r += kBlock) {
        double* ar = A + static_cast<size_t>(r) * KP;
        for (int k = K - 1; k >= 0; --k) {
            double acc = 0.0;
            for (int m = 0; m <= k; ++m) acc = fma(ar[m], X[k * GP + m], acc);
            ar[k] = acc;
        }
        for (int k = 0; k < K; ++k) {
            double acc = 0.0;
            for (int m = k; m < K; ++m) acc = fma(ar[m], X[m * GP + k], acc);
            ar[k] = acc;
        }
    }
    __syncthreads();
    for (int e = tid; e < S * K; e += kBlock) {
        const int k = e / S, r = e - k * S;
        pt[e] = static_cast<T>(A[r * KP + k]);
    }
}

hipError_t launch_lsq_pinv(bool dbl, const void* omt, const void* q, int I, int S, int K, void* pt,
                           uint32_t* flags, hipStream_t s) {
    if (K < 1 || K > 64 || S < K || I < 1) return hipErrorInvalidValue;
    const size_t lds = lsq_lds_doubles(S, K) * sizeof(double);
    if (lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
#define RH_LSQ_CASE(KBV)                                                                         \
    case KBV:                                                                                    \
        if (dbl)                                                                                 \
            hipLaunchKernelGGL((k_lsq_pinv<KBV, double>), dim3(1), dim3(kBlock), lds, s,          \
                               static_cast<const double*>(omt), static_cast<const double*>(q), I, \
                               S, K, static_cast<double*>(pt), flags);                           \
        else                                                                                     \
            hipLaunchKernelGGL((k_lsq_pinv<KBV, float>), dim3(1), dim3(kBlock), lds, s,           \
                               static_cast<const float*>(omt), static_cast<const float*>(q), I,   \
                               S, K, static_cast<float*>(pt), flags);                            \
        break;
    switch ((K + 7) & ~7) {
        RH_LSQ_CASE(8)
        RH_LSQ_CASE(16)
        RH_LSQ_CASE(24)
        RH_LSQ_CASE(32)
        RH_LSQ_CASE(40)
        RH_LSQ_CASE(48)
        RH_LSQ_CASE(56)
        RH_LSQ_CASE(64)
        default:
            return hipErrorInvalidValue;
    }
#undef RH_LSQ_CASE
    return hipGetLastError();
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

// ---------------------------------------------------------------------------
// Symmetric EVD by Householder tridiagonalisation, bisection on Sturm counts
// and inverse iteration (Golub & Van Loan, Matrix Computations, 8.3.1 and
// 8.4; the bisection / inverse-iteration scheme of LAPACK's dstebz and
// dstein), for K <= 64 in one workgroup.  Jacobi rounds on this CU are bound
// by LDS instruction issue; here the sequential parts live in registers.
//   1. wave 0, lane i = row i of A (registers): for k = 0..K-3 a reflector
//      H_k = I - tau v v^T (v_{k+1} = 1) zeroes A(k+2:, k); p = tau A v and
//      w = p - (tau/2)(p^T v) v give A <- A - v w^T - w v^T.  d, e to LDS,
//      v and tau kept for the back-transformation (the update is applied as
//      A - v p^T - (p - tau (p^T v) v) v^T, the same matrix).
//   2. all threads, seven lanes per eigenvalue j (ascending): each lane counts
//      the eigenvalues below one of the seven interior points of an 8-way
//      split of [lo, hi) (Sturm count: negative pivots of T - x I, pivots
//      kept away from zero by pivmin), a wave ballot counts the group's
//      points with at most j eigenvalues below, and the group keeps the
//      eighth that holds lambda_j; 18 steps take the Gershgorin interval to
//      about 1e-16 of norm(T).
//   3. wave 0, lane j = eigenvalue j: inverse iteration from a fixed
//      pseudo-random unit start, each step a solve with T - lambda_j I
//      factored by Gaussian elimination with row interchanges (the factor
//      kept in LDS, the vector in registers), normalised, then Gram-Schmidt
//      against the earlier vectors of its cluster; a second (third) step only
//      while some vector grew by less than 1e11 / norm(T), i.e. its residual
//      is above 1e-11 norm(T).  With the shift accurate to rounding one solve
//      leaves the other directions at about eps norm(T) / gap, so only
//      eigenvalues closer than 1e-4 norm(T) form a cluster (dstein's 1e-3
//      would also sweep in well separated ones).
//   4. wave 0: z <- H_0 ... H_{K-3} z.
//   5. convergence check on T: the residual norm(T z - lambda z) against
//      1e-10 norm(T), and the orthogonality of each vector to its neighbours
//      and its cluster against 1e-10; a miss sets RHOSVD_FLAG_EVD_NOCONV.
// Outputs: v (K x K column-major, column r the eigenvector of the r-th largest
// eigenvalue) and lambda (descending), or with FACTOR the factor step on them
// in the same launch.  LDS: evd_tri_lds_doubles(K), then the eigenpairs.
// ---------------------------------------------------------------------------
constexpr int kTriMaxIters = 3;    // solves of inverse iteration, while some vector grows too little
constexpr int kBisectSteps = 18;   // the Gershgorin interval to ~1e-16 norm(T)
constexpr double kClusterGap = 1e-4;  // Gram-Schmidt within gaps below this, relative to norm(T)
constexpr int kTriP = RHOSVD_MAX_K / 2;   // row pitch of the LDS vectors (64 >= K)

__host__ __device__ inline size_t evd_tri_lds_doubles(int K) {
    return static_cast<size_t>(kTriP) * kTriP + 3 * static_cast<size_t>(K) * kWave + 6 * kTriP;
}

// value of a[idx] for a uniform runtime idx (registers cannot be indexed):
// four independent select chains, then one of the four by idx & 3
template <int KB>
__device__ __forceinline__ double pick(const double (&a)[KB], int idx) {
    double r[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < KB; ++c) r[c & 3] = (c == idx) ? a[c] : r[c & 3];
    const int m = idx & 3;
    return m == 0 ? r[0] : (m == 1 ? r[1] : (m == 2 ? r[2] : r[3]));
}

// pick over the entries J0 .. KB - 1 only (idx >= J0)
template <int KB, int J0>
__device__ __forceinline__ double pick_from(const double (&a)[KB], int idx) {
    double r[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = J0; c < KB; ++c) r[c & 3] = (c == idx) ? a[c] : r[c & 3];
    const int m = idx & 3;
    return m == 0 ? r[0] : (m == 1 ? r[1] : (m == 2 ? r[2] : r[3]));
}

// Sum over the wave, the same value in every lane: butterflies inside quads
// and rows of 16 on DPP lane moves (no LDS), then the four row sums.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                                       static_cast<unsigned>(lo)));
}

__device__ __forceinline__ double wave_total(double v) {
    v += dpp_d<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x124>(v);   // row_ror:4
    v += dpp_d<0x128>(v);   // row_ror:8
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// ---------------------------------------------------------------------------
// Householder QR of Y (I x K column-major FP64, K <= I <= 16 RPL, K <= 64) in
// one workgroup of W waves (Golub & Van Loan, Matrix Computations, 5.2.1, with
// the backward accumulation of Q of 5.1.6).  Column c = 4 W s + W g + w lives
// in wave w, lane group g (lanes 16 g .. 16 g + 15, one DPP row) and register
// slot s; lane 16 g + t holds its rows t + 16 r (r < RPL = 16 or 32).  A
// column's dot product is then one reduction within a DPP row, and one
// reduction serves the four columns of a slot in a wave together.  Column
// step j: its group forms the reflector H_j = I - tau v v^T (v_j = A(j,j) -
// alpha, v_i = A(i,j) below, alpha = -sign(A(j,j)) norm(A(j:,j))) and
// broadcasts v through LDS; every wave applies H_j to its columns past j.  The
// loops over slots and 16-column sub-blocks are unrolled, the inner one over
// 16 columns is not, so register indices are constants (row j sits in
// register j / 16) and the slots before the current one drop out at compile
// time.  Then Q = H_0 ... H_{K-1} [I_K; 0] backwards, each wave on its own
// columns from the stored reflectors (no barriers), and columns with
// alpha < 0 negated: diag(R) >= 0, the same Q as CholeskyQR for full-rank Y.
// One barrier per column step; LDS: K x 16 RPL doubles of reflectors.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double row16_total(double v) {
    v += dpp_d<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x124>(v);   // row_ror:4
    v += dpp_d<0x128>(v);   // row_ror:8
    return v;
}

template <int W, int NS, int RPL>
__device__ __forceinline__ void hqr_body(const double* __restrict__ y, int I, int K,
                                         double* __restrict__ q64, void* q_out, int dbl) {
    extern __shared__ __align__(16) double shd[];
    constexpr int VP = 16 * RPL;                   // rows held: 16 lanes x RPL
    constexpr int SW = 4 * W;                      // columns per slot
    constexpr int SB = SW / 16;                    // 16-column sub-blocks of a slot
    static_assert(W >= 4 && W % 4 == 0, "a slot holds whole 16-column sub-blocks");
    double* V = shd;                               // reflector j at V[j * VP + row]
    __shared__ double tau_s[RHOSVD_MAX_K], alpha_s[RHOSVD_MAX_K];
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    const int g = lane >> 4, t = lane & 15;
    const int cw = W * g + wave;                   // column within a slot
    double a[NS][RPL];
#pragma unroll
    for (int m = 0; m < NS; ++m)
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int c = SW * m + cw, row = t + 16 * r;
            a[m][r] = (c < K && row < I) ? y[static_cast<size_t>(c) * I + row] : 0.0;
        }
    // column step j = SW m + 16 rb + jc (row j sits in register SB m + rb of
    // lane jc of its group: a compile-time index)
#pragma unroll
    for (int m = 0; m < NS; ++m) {
#pragma unroll
        for (int rb = 0; rb < SB; ++rb) {
#pragma unroll 1
            for (int jc = 0; jc < 16; ++jc) {
                const int js = 16 * rb + jc;           // column within the slot: W og + ow
                const int j = SW * m + js;
                if (j >= K) break;                     // uniform
                const int ow = js % W, og = js / W;
                if (wave == ow) {
                    double s4[4] = {0.0, 0.0, 0.0, 0.0};     // four independent chains
#pragma unroll
                    for (int r = 0; r < RPL; ++r) {
                        const double x = t + 16 * r >= j ? a[m][r] : 0.0;
                        s4[r & 3] = fma(x, x, s4[r & 3]);
                    }
                    const double s2 = (s4[0] + s4[1]) + (s4[2] + s4[3]);
                    const double n2 = readlane_d(row16_total(s2), 16 * og);
                    const double ajj = readlane_d(a[m][SB * m + rb], 16 * og + jc);
                    const double alpha = (ajj > 0.0 ? -1.0 : 1.0) * sqrt(n2);
                    const double v0 = ajj - alpha;
                    const double vn2 = fma(v0, v0, n2 - ajj * ajj);
                    const double tau = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
                    if (g == og) {
#pragma unroll
                        for (int r = 0; r < RPL; ++r) {
                            const int row = t + 16 * r;
                            V[j * VP + row] = row == j ? v0 : (row > j ? a[m][r] : 0.0);
                        }
                    }
                    if (lane == 0) {
                        tau_s[j] = tau;
                        alpha_s[j] = alpha;
                    }
                }
                __syncthreads();
                const double tau = tau_s[j];
                double v[RPL];
#pragma unroll
                for (int r = 0; r < RPL; ++r) v[r] = V[j * VP + t + 16 * r];
                // columns past j: every later slot, and in slot m the columns
                // after js (columns past K are zero and stay zero)
#pragma unroll
                for (int mm = m; mm < NS; ++mm) {
                    double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int r = 0; r < RPL; ++r) d4[r & 3] = fma(v[r], a[mm][r], d4[r & 3]);
                    double d = row16_total((d4[0] + d4[1]) + (d4[2] + d4[3])) * tau;
                    if (mm == m) d = cw > js ? d : 0.0;
#pragma unroll
                    for (int r = 0; r < RPL; ++r) a[mm][r] = fma(-d, v[r], a[mm][r]);
                }
            }
        }
    }
    __syncthreads();
    // Q backwards: H_j changes only the columns c >= j
    double q[NS][RPL];
#pragma unroll
    for (int m = 0; m < NS; ++m)
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int c = SW * m + cw;
            q[m][r] = (c < K && t + 16 * r == c) ? 1.0 : 0.0;
        }
#pragma unroll
    for (int m = NS - 1; m >= 0; --m) {
#pragma unroll
        for (int rb = SB - 1; rb >= 0; --rb) {
#pragma unroll 1
            for (int jc = 15; jc >= 0; --jc) {
                const int js = 16 * rb + jc;
                const int j = SW * m + js;
                if (j >= K) continue;
                const double tau = tau_s[j];
                double v[RPL];
#pragma unroll
                for (int r = 0; r < RPL; ++r) v[r] = V[j * VP + t + 16 * r];
#pragma unroll
                for (int mm = m; mm < NS; ++mm) {
                    double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int r = 0; r < RPL; ++r) d4[r & 3] = fma(v[r], q[mm][r], d4[r & 3]);
                    double d = row16_total((d4[0] + d4[1]) + (d4[2] + d4[3])) * tau;
                    if (mm == m) d = cw >= js ? d : 0.0;
#pragma unroll
                    for (int r = 0; r < RPL; ++r) q[mm][r] = fma(-d, v[r], q[mm][r]);
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < NS; ++m) {
        const int c = SW * m + cw;
        if (c < K) {
            const double sg = alpha_s[c] < 0.0 ? -1.0 : 1.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int row = t + 16 * r;
                if (row < I) {
                    const size_t e = static_cast<size_t>(c) * I + row;
                    const double val = sg * q[m][r];
                    q64[e] = val;
                    if (dbl)
                        static_cast<double*>(q_out)[e] = val;
                    else
                        static_cast<float*>(q_out)[e] = static_cast<float>(val);
                }
            }
        }
    }
}

// W = 4 waves: measured at I = 200, K = 35, 44 us against 48 (8 waves) and
// 50 (16 waves): the column steps are bound by the reflector's broadcast and
// the barrier, which more waves make slower, not by the updates they share
template <int W, int NS, int RPL>
__global__ __launch_bounds__(64 * W) void k_hqr(const double* __restrict__ y, int I, int K,
                                                double* __restrict__ q64, void* q_out, int dbl) {
    hqr_body<W, NS, RPL>(y, I, K, q64, q_out, dbl);
}

// One QR per workgroup from a device table (many small problems in one launch).
template <int NS, int RPL>
__global__ __launch_bounds__(kBlock) void k_hqr_batch(const QrJob* __restrict__ jobs) {
    const QrJob j = jobs[blockIdx.x];
    hqr_body<kBlock / kWave, NS, RPL>(j.y, j.I, j.K, j.q64, j.q_out, j.dbl);
}

static hipError_t launch_hqr(const double* y, int I, int K, bool dbl, void* q_out, double* q64,
                             hipStream_t s) {
    constexpr int W = kBlock / kWave;
    const int rpl = I <= 256 ? 16 : 32;
    const size_t lds = static_cast<size_t>(K) * 16 * rpl * sizeof(double);
    const int d = dbl ? 1 : 0;
#define RH_HQR_CASE(N, R)                                                                           \
    case N:                                                                                         \
        hipLaunchKernelGGL((k_hqr<W, N, R>), dim3(1), dim3(kBlock), lds, s, y, I, K, q64, q_out, d); \
        break;
    if (rpl == 16) {
        switch ((K + 15) / 16) {
            RH_HQR_CASE(1, 16)
            RH_HQR_CASE(2, 16)
            RH_HQR_CASE(3, 16)
            RH_HQR_CASE(4, 16)
            default:
                return hipErrorInvalidValue;
        }
    } else {
        switch ((K + 15) / 16) {
            RH_HQR_CASE(1, 32)
            RH_HQR_CASE(2, 32)
            default:
                return hipErrorInvalidValue;
        }
    }
#undef RH_HQR_CASE
    return hipGetLastError();
}

hipError_t launch_hqr_fwd(const double* y, int I, int K, bool dbl, void* q_out, double* q64,
                          hipStream_t s) {
    return launch_hqr(y, I, K, dbl, q_out, q64, s);
}

// Factor step (Algorithm 1 steps 6-7) on the sorted eigenpairs of the Gram:
// U = Q V[:, :R] (V = identity when use_v == 0), canonical signs (each
// column's largest-magnitude entry positive, the lowest row on ties),
// M = V_R with the same signs (K x R), sigma = sqrt(max(lambda, 0))[:R].
// Q (I x K column-major, T) is staged row-major with pitch K16 + 1 (zero padded
// to I16 rows) at Qs (LDS, or global scratch when it does not fit); U is
// formed on the f64 matrix cores in place of Q, one 16-row block per wave at
// a time.  Vs: K x K column-major (LDS), lamS: K (LDS).
// Elements tid + u kBlock (u < QN) of Q, loaded early in the EVD kernel so
// that their latency is hidden behind the tridiagonal phases: 32 per thread,
// 8 for K > 48, whose eigenvector phases need the registers.
template <int KB>
constexpr int q_prefetch() { return KB > 48 ? 8 : 32; }

template <typename T, int QN>
__device__ void factor_step(int K, int K16, int I, int I16, int R, int use_v, const double* Vs,
                            const double* lamS, const T* __restrict__ q, double* Qs,
                            T* __restrict__ u_out, T* __restrict__ m_out,
                            double* __restrict__ sigma, const T (&qpre)[QN]) {
    __shared__ double sgn[RHOSVD_MAX_K];
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    // odd row pitch: a column walk (consecutive rows, one column) spreads
    // over the LDS banks instead of hitting the same two
    const int QP = K16 + 1;
    // the padding first (rows I.. as one range, then columns K.. of each
    // row), then Q in its own column-major order (coalesced): the first
    // round from the registers loaded early, later ones (past QN kBlock
    // elements) with QN loads in flight per thread
    for (int e = I * QP + tid; e < I16 * QP; e += kBlock) Qs[e] = 0.0;
    for (int i = tid; i < I; i += kBlock)
        for (int k = K; k < QP; ++k) Qs[i * QP + k] = 0.0;
    const int n = I * K;
    for (int e0 = tid; e0 < n; e0 += QN * kBlock) {
        T v[QN];
#pragma unroll
        for (int u = 0; u < QN; ++u) {
            const int e = e0 + u * kBlock;
            v[u] = e0 == tid ? qpre[u] : q[e < n ? e : n - 1];
        }
        int k = e0 / I, i = e0 - k * I;
        const int dk = kBlock / I, di = kBlock - dk * I;
#pragma unroll
        for (int u = 0; u < QN; ++u) {
            if (e0 + u * kBlock < n) Qs[i * QP + k] = static_cast<double>(v[u]);
            i += di;
            k += dk;
            if (i >= I) {
                i -= I;
                ++k;
            }
        }
    }
    __syncthreads();
    {
        // V_R's fragments stay in registers for all row blocks (K16 <= 64,
        // R <= 64); each row block loads its Q fragments at once
        const int m = lane & 15, kq = lane >> 4;
        const int nib = I16 >> 4, nrb = (R + 15) >> 4, nst = K16 >> 2;
        double vb[4][16];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int st = 0; st < 16; ++st) {
                const int k = 4 * st + kq, rcol = 16 * rb + m;
                double b = 0.0;
                if (rb < nrb && st < nst && rcol < R && k < K)
                    b = use_v ? Vs[rcol * K + k] : (k == rcol ? 1.0 : 0.0);
                vb[rb][st] = b;
            }
        for (int ib = wave; ib < nib; ib += kBlock / kWave) {
            const double* qa = Qs + (16 * ib + m) * QP + kq;
            double a[16];
#pragma unroll
            for (int st = 0; st < 16; ++st) a[st] = st < nst ? qa[4 * st] : 0.0;
            f64x4 acc[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                acc[rb] = zero4<f64x4>();
                if (rb < nrb) {
#pragma unroll
                    for (int st = 0; st < 16; ++st)
                        if (st < nst) acc[rb] = Mma<double>::step(a[st], vb[rb][st], acc[rb]);
                }
            }
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                if (rb < nrb) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * ib + Mma<double>::row(kq, r), col = 16 * rb + m;
                        if (col < R) Qs[row * QP + col] = acc[rb][r];
                    }
                }
            }
        }
    }
    __syncthreads();
    {
        // canonical signs, every column at once: four consecutive threads per
        // column (R <= 64), each scanning rows sub, sub + 4, ... in ascending
        // order (a strict > keeps the lowest row among equal magnitudes), then
        // the quad combined with the same rule
        const int r = tid >> 2, sub = tid & 3;
        double best = -1.0;
        int bi = 0x7fffffff;
        if (r < R) {
            for (int i = sub; i < I; i += 4) {
                const double a = fabs(Qs[i * QP + r]);
                if (a > best) {
                    best = a;
                    bi = i;
                }
            }
        }
#pragma unroll
        for (int o = 1; o < 4; o <<= 1) {
            const double ob = __shfl_xor(best, o, kWave);
            const int oi = __shfl_xor(bi, o, kWave);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (sub == 0 && r < R) sgn[r] = (Qs[bi * QP + r] < 0.0) ? -1.0 : 1.0;
    }
    __syncthreads();
    for (int e = tid; e < I * R; e += kBlock) {
        const int r = e / I, i = e - r * I;
        u_out[e] = static_cast<T>(sgn[r] * Qs[i * QP + r]);
    }
    for (int e = tid; e < K * R; e += kBlock) {
        const int r = e / K, k = e - r * K;
        const double vv = use_v ? Vs[r * K + k] : (k == r ? 1.0 : 0.0);
        m_out[e] = static_cast<T>(sgn[r] * vv);
    }
    if (sigma)
        for (int r = tid; r < R; r += kBlock) sigma[r] = sqrt(fmax(lamS[r], 0.0));
}

// Start vector of inverse iteration: entries in [-1, 1) from a 32-bit hash
// of (i, j) (an integer mixer of the murmur finaliser kind).
__device__ __forceinline__ double start_entry(int i, int j) {
    uint32_t h = static_cast<uint32_t>(i) * 0x9E3779B1u ^ (static_cast<uint32_t>(j) + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    return static_cast<double>(h) * (2.0 / 4294967296.0) - 1.0;
}

// The code keeps the outer loops rolled: only loops over the register arrays
// (length KB) are unrolled, so the kernel stays small enough for the
// instruction cache.  LDS vectors have pitch kTriP and are zero past K, so
// those loops need no bounds.
template <int KB, typename T, bool FACTOR>
__device__ __forceinline__ void evd_tri_body(const double* __restrict__ cin, int K,
                                                   double* __restrict__ v_out,
                                                   double* __restrict__ lam_out, uint32_t* flags,
                                                   const T* __restrict__ q, int I, int R, int use_v,
                                                   T* __restrict__ u_out, T* __restrict__ m_out,
                                                   double* __restrict__ sigma,
                                                   double* __restrict__ qwork, int staged) {
    extern __shared__ __align__(16) double shd[];
    double* hv = shd;                                  // kTriP x kTriP: row k = v of H_k
    double* lu = hv + kTriP * kTriP;                   // [3][K][64] factor of T - lambda I, per lane
    double* zs = lu;                                   // K x kTriP vectors (between solves)
    double* tau = lu + 3 * static_cast<size_t>(K) * kWave;
    double* dd = tau + kTriP;
    double* ee = dd + kTriP;
    double* lam = ee + kTriP;
    double* bc = lam + kTriP;                          // broadcast of v
    double* bw = bc + kTriP;                           // broadcast of w
    // once the tridiagonal phases are done (wave 0 last reads hv in the
    // back-transformation, then writes the eigenpairs), the start of the
    // region holds the sorted eigenpairs and Q is staged after them
    const int K16 = (K + 15) & ~15, I16 = (I + 15) & ~15;
    double* Vs = shd;                                  // K x K, column r = r-th largest
    double* lamS = Vs + static_cast<size_t>(K) * K;    // K, descending
    double* Qst = lamS + K + (K & 1);                  // I16 x (K16 + 1) when staged
    __shared__ double stats[2];                        // norm(T), pivmin
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    for (int e = tid; e < kTriP * kTriP; e += kBlock) hv[e] = 0.0;
    for (int e = tid; e < 6 * kTriP; e += kBlock) tau[e] = 0.0;
    __syncthreads();

    // ---- 1. tridiagonalisation (wave 0) ----
    if (wave == 0) {
        double a[KB];
        const int li = lane < K ? lane : 0;
#pragma unroll
        for (int c = 0; c < KB; ++c) a[c] = (lane < K && c < K) ? cin[static_cast<size_t>(c) * K + li] : 0.0;
        // Step k touches only rows and columns past k (v and p vanish at
        // indices <= k), so the steps run in segments of eight whose column
        // loops start at the segment's first step (J0 <= k).
        auto step = [&](auto J0c, int k) __attribute__((always_inline)) {
            constexpr int J0 = decltype(J0c)::value;
            const double ak = pick_from<KB, J0>(a, k);
            const double x = lane > k ? ak : 0.0;                 // A(k+1:, k)
            const double akk = readlane_d(ak, k);
            const double x1 = readlane_d(ak, k + 1);
            const double tail = wave_total(lane > k + 1 ? x * x : 0.0);
            double beta = x1, t = 0.0, scale = 0.0;
            if (tail > 0.0) {
                const double nrm = sqrt(fma(x1, x1, tail));
                beta = x1 >= 0.0 ? -nrm : nrm;
                t = (beta - x1) / beta;
                scale = 1.0 / (x1 - beta);
            }
            const double v = lane == k + 1 ? 1.0 : (lane > k + 1 ? x * scale : 0.0);
            if (lane < K) hv[k * kTriP + lane] = v;
            if (lane == 0) {
                tau[k] = t;
                dd[k] = akk;
                ee[k] = beta;
            }
            if (t != 0.0) {
                // v and p broadcast through LDS (zero past K), read in pairs
                if (lane < K) bc[lane] = v;
                double pq[4] = {0.0, 0.0, 0.0, 0.0};   // four independent chains
#pragma unroll
                for (int j = J0; j < KB; j += 2) {
                    const double2 c2 = *reinterpret_cast<const double2*>(bc + j);
                    pq[j & 3] = fma(a[j], c2.x, pq[j & 3]);
                    pq[(j + 1) & 3] = fma(a[j + 1], c2.y, pq[(j + 1) & 3]);
                }
                const double pv = (pq[0] + pq[1]) + (pq[2] + pq[3]);
                const double p = lane > k ? t * pv : 0.0;
                // A - v w^T - w v^T with w = p - kk v equals
                // A - v p^T - (p - 2 kk v) v^T: p is broadcast while the sum
                // for kk is formed
                if (lane < K) bw[lane] = p;
                const double kk = 0.5 * t * wave_total(p * v);
                const double u = fma(-2.0 * kk, v, p);
#pragma unroll
                for (int j = J0; j < KB; j += 2) {
                    const double2 c2 = *reinterpret_cast<const double2*>(bc + j);
                    const double2 w2 = *reinterpret_cast<const double2*>(bw + j);
                    a[j] = fma(-v, w2.x, fma(-u, c2.x, a[j]));
                    a[j + 1] = fma(-v, w2.y, fma(-u, c2.y, a[j + 1]));
                }
            }
        };
        auto seg = [&](auto J0c) __attribute__((always_inline)) {
            constexpr int J0 = decltype(J0c)::value;
            if constexpr (J0 < KB) {
                const int kend = J0 + 8 < K - 2 ? J0 + 8 : K - 2;
#pragma unroll 1
                for (int k = J0; k < kend; ++k) step(J0c, k);
            }
        };
        seg(std::integral_constant<int, 0>{});
        seg(std::integral_constant<int, 8>{});
        seg(std::integral_constant<int, 16>{});
        seg(std::integral_constant<int, 24>{});
        seg(std::integral_constant<int, 32>{});
        seg(std::integral_constant<int, 40>{});
        seg(std::integral_constant<int, 48>{});
        seg(std::integral_constant<int, 56>{});
        if (K >= 2) {
            const double d0 = readlane_d(pick(a, K - 2), K - 2);
            const double d1 = readlane_d(pick(a, K - 1), K - 1);
            const double e0 = readlane_d(pick(a, K - 2), K - 1);
            if (lane == 0) {
                dd[K - 2] = d0;
                dd[K - 1] = d1;
                ee[K - 2] = e0;
            }
        } else {
            const double d0 = readlane_d(a[0], 0);
            if (lane == 0) dd[0] = d0;
        }
        if (lane == 0) {
            // Gershgorin radius as the norm bound; pivmin as in dstebz
            double tn = 0.0, emax = 1.0;
            for (int i = 0; i < K; ++i) {
                const double el = i > 0 ? fabs(ee[i - 1]) : 0.0, er = i < K - 1 ? fabs(ee[i]) : 0.0;
                tn = fmax(tn, fabs(dd[i]) + el + er);
                if (i < K - 1) emax = fmax(emax, ee[i] * ee[i]);
            }
            stats[0] = tn;
            stats[1] = 2.2250738585072014e-308 * emax;
        }
    }
    // the factor step's first round of Q (waves 1-3 load it while wave 0
    // tridiagonalises; used only after the last phase)
    constexpr int QN = q_prefetch<KB>();
    T qpre[QN];
    if constexpr (FACTOR) {
        const int n = I * K;
#pragma unroll
        for (int u = 0; u < QN; ++u) {
            const int e = tid + u * kBlock;
            qpre[u] = q[e < n ? e : n - 1];
        }
    }
    __syncthreads();

    // ---- 2. eigenvalues by multisection (all threads; 7 lanes per eigenvalue) ----
    {
        const double tn = stats[0], pivmin = stats[1];
        // lanes 7 q .. 7 q + 6 of wave w (q < 9) own eigenvalue jb + 9 w + q
        const int grpq = lane / 7, sub = lane - 7 * grpq;
        const uint64_t gmask = grpq < 9 ? (0x7FULL << (7 * grpq)) : 0ULL;
        // rows past K: d huge and e zero keep their pivots positive, so they
        // never count and need no masking
        double d[KB], e2[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            d[i] = i < K ? dd[i] : 1e300;
            e2[i] = ee[i] * ee[i];                 // ee is zero past K - 2
        }
        auto multisect = [&](double& lo, double& hi, int j, int steps) {
#pragma unroll 1
            for (int st = 0; st < steps; ++st) {
                // point sub + 1 of the 8-way split (point 8 is hi itself)
                const double h = (hi - lo) * 0.125;
                const double xa = lo + (sub + 1) * h;
                double qa = d[0] - xa;
                qa = fabs(qa) < pivmin ? -pivmin : qa;
                int ca = qa < 0.0;
#pragma unroll
                for (int i = 1; i < KB; ++i) {
                    qa = fma(-e2[i - 1], rcp_nr(qa), d[i] - xa);
                    qa = fabs(qa) < pivmin ? -pivmin : qa;
                    ca += qa < 0.0 ? 1 : 0;
                }
                // how many of the group's seven points have at most j
                // eigenvalues below them
                const int nle = __popcll(__ballot(ca <= j) & gmask);
                const double nlo = lo + nle * h;
                hi = nle == 7 ? hi : lo + (nle + 1) * h;
                lo = nlo;
            }
        };
        // eigenvalue j of round r: jb = 36 r (K <= 64: two rounds at most)
        constexpr int kPerRound = 9 * (kBlock / kWave);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int j = kPerRound * r + 9 * wave + grpq;
            double lo = -tn - 4.0 * pivmin - 2.2e-16 * 4.0 * K * tn - 1e-300;
            double hi = tn + 4.0 * pivmin + 2.2e-16 * 4.0 * K * tn + 1e-300;
            if (kPerRound * r < K) {
                multisect(lo, hi, j, kBisectSteps);
                if (sub == 0 && grpq < 9 && j < K) lam[j] = 0.5 * (lo + hi);
            }
        }
    }
    __syncthreads();

    // ---- 3-4. eigenvectors (wave 0, lane j = eigenvalue j); the check (5)
    // runs in wave 1 beside the back-transformation in wave 0 ----
    const double tn = stats[0];
    const double ctol = kClusterGap * tn;                      // cluster distance
    const int jl = lane < K ? lane : K - 1;
    const double lj = lam[jl];
    // cluster id: the number of gaps above ctol below this eigenvalue;
    // mates: bit m set when eigenvalue m has a later member of its cluster
    int cid = 0;
    for (int q = 1; q <= jl; ++q) cid += (lam[q] - lam[q - 1] > ctol) ? 1 : 0;
    const bool has_mate = lane + 1 < K && (lam[lane + 1] - lam[lane] <= ctol);
    const uint64_t mates = __ballot(has_mate);
    double z[KB];
    if (wave == 0) {
        const double tiny = 2.2e-16 * fmax(tn, 1e-300);      // pivot floor of T - lambda I
        double* u1 = lu;
        double* u2 = lu + K * kWave;
        double* u3 = lu + 2 * K * kWave;
        {
            double s2 = 0.0;
#pragma unroll
            for (int i = 0; i < KB; ++i) {
                z[i] = i < K ? start_entry(i, jl) : 0.0;
                s2 = fma(z[i], z[i], s2);
            }
            const double r = rsq_nr(s2);
#pragma unroll
            for (int i = 0; i < KB; ++i) z[i] *= r;
        }
        // a solve of (T - lambda I) x = z with norm(z) = 1 leaves z' = x / norm(x)
        // with residual norm(T z' - lambda z') = 1 / norm(x): the vector has
        // converged when norm(x) >= 1e11 / norm(T)
        const double grow2 = 1e22 / fmax(tn * tn, 1e-300);
#pragma unroll 1
        for (int it = 0; it < kTriMaxIters; ++it) {
            // forward: elimination with row interchanges (branch-free), the
            // same operations applied to z; rows past K are left alone
            double ca = dd[0] - lj, cb = ee[0], cd = 0.0;
#pragma unroll
            for (int i = 0; i < KB - 1; ++i) {
                const bool in = i < K - 1;
                const double ci = ee[i];                 // sub-diagonal of row i+1
                const double an = dd[i + 1] - lj;        // diagonal of row i+1
                const double bn = ee[i + 1];             // super-diagonal of row i+1
                const bool swap = fabs(ca) < fabs(ci);
                const double pa = fabs(ca) < tiny ? (ca < 0.0 ? -tiny : tiny) : ca;
                const double piv = swap ? ci : pa;
                const double l = (swap ? ca : ci) * rcp_nr(piv);
                const double zi = z[i], zn = z[i + 1];
                if (in) {
                    u1[i * kWave + lane] = piv;
                    u2[i * kWave + lane] = swap ? an : cb;
                    u3[i * kWave + lane] = swap ? bn : cd;
                    z[i] = swap ? zn : zi;
                    z[i + 1] = swap ? fma(-l, zn, zi) : fma(-l, zi, zn);
                    const double na = swap ? fma(-l, an, cb) : fma(-l, cb, an);
                    cb = swap ? fma(-l, bn, cd) : fma(-l, cd, bn);
                    ca = na;
                    cd = 0.0;
                }
            }
            {
                const double pa = fabs(ca) < tiny ? (ca < 0.0 ? -tiny : tiny) : ca;
                u1[(K - 1) * kWave + lane] = pa;
                u2[(K - 1) * kWave + lane] = 0.0;
                u3[(K - 1) * kWave + lane] = 0.0;
            }
            // back substitution, from the last row up
            double z1 = 0.0, z2 = 0.0;   // z[i + 1], z[i + 2]
#pragma unroll
            for (int i = KB - 1; i >= 0; --i) {
                if (i < K) {
                    const double r = fma(-u2[i * kWave + lane], z1, fma(-u3[i * kWave + lane], z2, z[i]));
                    z[i] = r * rcp_nr(u1[i * kWave + lane]);
                    z2 = z1;
                    z1 = z[i];
                }
            }
            double nn = 0.0;
#pragma unroll
            for (int i = 0; i < KB; ++i) nn = fma(z[i], z[i], nn);
            const bool conv = !(lane < K) || nn >= grow2;
            double inv = rsq_nr(nn);
#pragma unroll
            for (int i = 0; i < KB; ++i) z[i] *= inv;
            // Gram-Schmidt within clusters, in ascending order: vector m is
            // final when its turn comes; the later members of its cluster
            // remove their component along it
            for (uint64_t mm = mates; mm != 0; mm &= mm - 1) {
                const int m = __builtin_ctzll(mm);                  // uniform
                if (lane == m) {
                    double s2 = 0.0;
#pragma unroll
                    for (int i = 0; i < KB; ++i) s2 = fma(z[i], z[i], s2);
                    const double r = rsq_nr(s2);
#pragma unroll
                    for (int i = 0; i < KB; ++i) {
                        z[i] *= r;
                        zs[m * kTriP + i] = z[i];
                    }
                }
                const bool mate = lane > m && lane < K && cid == __builtin_amdgcn_readlane(cid, m);
                double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int i = 0; i < KB; ++i) d4[i & 3] = fma(zs[m * kTriP + i], z[i], d4[i & 3]);
                const double dot = (d4[0] + d4[1]) + (d4[2] + d4[3]);
                if (mate) {
#pragma unroll
                    for (int i = 0; i < KB; ++i) z[i] = fma(-dot, zs[m * kTriP + i], z[i]);
                }
            }
            nn = 0.0;
#pragma unroll
            for (int i = 0; i < KB; ++i) nn = fma(z[i], z[i], nn);
            inv = rsq_nr(nn);
#pragma unroll
            for (int i = 0; i < KB; ++i) z[i] *= inv;
            if (__ballot(!conv) == 0ull) break;           // wave-uniform
        }
        // the vectors for the check
        if (lane < K) {
#pragma unroll
            for (int i = 0; i < KB; ++i) zs[lane * kTriP + i] = z[i];
        }
    }
    __syncthreads();
    if (wave == 1) {
        // convergence check: residual norm(T z - lambda z) against norm(T),
        // and orthogonality to the neighbouring vectors and to the cluster's
        // (vectors of eigenvalues further apart than the cluster distance
        // are orthogonal to about eps norm(T) / gap by construction)
        double zc[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) zc[i] = zs[jl * kTriP + i];
        double tz[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            double t = 0.0;
            if (i < K) {
                t = dd[i] * zc[i];
                if (i > 0) t = fma(ee[i - 1], zc[i - 1], t);
                if (i + 1 < KB && i + 1 < K) t = fma(ee[i], zc[i + 1], t);
            }
            tz[i] = t;
        }
        double res = 0.0;
#pragma unroll
        for (int i = 0; i < KB; ++i) res = fmax(res, fabs(fma(-lj, zc[i], tz[i])));
        // cluster of this eigenvalue: [cs, ce] from the mates mask
        int cs = jl, ce = jl;
        while (cs > 0 && ((mates >> (cs - 1)) & 1ull)) --cs;
        while (ce + 1 < K && ((mates >> ce) & 1ull)) ++ce;
        const int mlo = cs < jl - 1 ? cs : (jl > 0 ? jl - 1 : 0);
        const int mhi = ce > jl + 1 ? ce : (jl + 1 < K ? jl + 1 : K - 1);
        double orth = 0.0;
#pragma unroll 1
        for (int m = mlo; m <= mhi; ++m) {
            double dq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < KB; i += 2) {
                const double2 c2 = *reinterpret_cast<const double2*>(zs + m * kTriP + i);
                dq[i & 3] = fma(c2.x, zc[i], dq[i & 3]);
                dq[(i + 1) & 3] = fma(c2.y, zc[i + 1], dq[(i + 1) & 3]);
            }
            const double dot = (dq[0] + dq[1]) + (dq[2] + dq[3]);
            orth = fmax(orth, fabs(dot - (m == jl ? 1.0 : 0.0)));
        }
        if (lane >= K) res = orth = 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            res = fmax(res, __shfl_xor(res, o, kWave));
            orth = fmax(orth, __shfl_xor(orth, o, kWave));
        }
        const bool bad = !(res <= 1e-10 * tn) || !(orth <= 1e-10);
        if (lane == 0 && flags && bad) atomicOr(flags, RHOSVD_FLAG_EVD_NOCONV);
    } else if (wave == 0) {
        // back-transformation z <- H_0 ... H_{K-3} z (rows of hv are zero
        // at indices <= k and past K)
#pragma unroll 1
        for (int k = K - 3; k >= 0; --k) {
            const double t = tau[k];
            double wq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < KB; ++i) wq[i & 3] = fma(hv[k * kTriP + i], z[i], wq[i & 3]);
            const double w = ((wq[0] + wq[1]) + (wq[2] + wq[3])) * t;
#pragma unroll
            for (int i = 0; i < KB; ++i) z[i] = fma(-w, hv[k * kTriP + i], z[i]);
        }
    }
    // the eigenpairs' region overlaps zs: written once the check is done
    __syncthreads();
    if (wave == 0 && lane < K) {
        const int col = K - 1 - lane;
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            if (i < K) {
                if (FACTOR)
                    Vs[static_cast<size_t>(col) * K + i] = z[i];
                else
                    v_out[static_cast<size_t>(col) * K + i] = z[i];
            }
        }
        if (FACTOR)
            lamS[col] = lj;
        else
            lam_out[col] = lj;
    }
    if constexpr (FACTOR) {
        __syncthreads();
        factor_step<T, QN>(K, K16, I, I16, R, use_v, Vs, lamS, q, staged ? Qst : qwork, u_out,
                           m_out, sigma, qpre);
    }
}

template <int KB, typename T, bool FACTOR>
__global__ __launch_bounds__(kBlock) void k_evd_tri(const double* __restrict__ cin, int K,
                                                   double* __restrict__ v_out,
                                                   double* __restrict__ lam_out, uint32_t* flags,
                                                   const T* __restrict__ q, int I, int R, int use_v,
                                                   T* __restrict__ u_out, T* __restrict__ m_out,
                                                   double* __restrict__ sigma,
                                                   double* __restrict__ qwork, int staged) {
    evd_tri_body<KB, T, FACTOR>(cin, K, v_out, lam_out, flags, q, I, R, use_v, u_out, m_out, sigma,
                                qwork, staged);
}

// EVD + factor step per workgroup from a device table.
template <int KB, typename T>
__global__ __launch_bounds__(kBlock) void k_evd_factor_batch(const EvdJob* __restrict__ jobs) {
    const EvdJob j = jobs[blockIdx.x];
    evd_tri_body<KB, T, true>(j.c, j.K, nullptr, nullptr, j.flags, static_cast<const T*>(j.q), j.I,
                              j.R, j.use_v, static_cast<T*>(j.u_out), static_cast<T*>(j.m_out),
                              j.sigma, j.qwork, j.staged);
}

// Dynamic LDS of k_evd_tri: the tridiagonal phases' region, reused by the
// factor step for the sorted eigenpairs (K x K + K doubles) and, when
// `staged`, Q after them.
static size_t evd_lds_bytes(int K, int64_t I, bool factor, bool staged) {
    const size_t K16 = (K + 15) & ~15, I16 = (I + 15) & ~static_cast<int64_t>(15);
    const size_t tri = evd_tri_lds_doubles(K);
    const size_t fac = factor ? static_cast<size_t>(K) * K + K + (K & 1) + (staged ? I16 * (K16 + 1) : 0) : 0;
    const size_t d = tri > fac ? tri : fac;
    return (d * sizeof(double) + 15) & ~static_cast<size_t>(15);
}

size_t evd_qwork_doubles(int K, int64_t I) {
    return static_cast<size_t>((I + 15) & ~static_cast<int64_t>(15)) * (((K + 15) & ~15) + 1);
}

template <typename T, bool FACTOR>
static hipError_t launch_evd_tri(const double* c, int K, double* v, double* lam, uint32_t* flags,
                                 const T* q, int I, int R, int use_v, T* u_out, T* m_out,
                                 double* sigma, double* qwork, int staged, size_t lds,
                                 hipStream_t s) {
#define RH_TRI_CASE(KBV)                                                                     \
    case KBV:                                                                                \
        hipLaunchKernelGGL((k_evd_tri<KBV, T, FACTOR>), dim3(1), dim3(kBlock), lds, s, c, K, \
                           v, lam, flags, q, I, R, use_v, u_out, m_out, sigma, qwork, staged); \
        break;
    switch ((K + 7) & ~7) {
        RH_TRI_CASE(8)
        RH_TRI_CASE(16)
        RH_TRI_CASE(24)
        RH_TRI_CASE(32)
        RH_TRI_CASE(40)
        RH_TRI_CASE(48)
        RH_TRI_CASE(56)
        RH_TRI_CASE(64)
        default:
            return hipErrorInvalidValue;
    }
#undef RH_TRI_CASE
    return hipGetLastError();
}

// EVD of C followed in the same launch by the factor step (U, M, sigma).
// u64: evd_qwork_doubles(K, I) doubles of device scratch, used when Q does
// not fit in LDS beside the eigenpairs.
hipError_t launch_evd_factor(bool dbl, const double* c, int K, uint32_t* flags, const void* q,
                             int64_t I, int R, int use_v, void* u_out, void* m_out, double* sigma,
                             double* u64, hipStream_t s) {
    if (K < 1 || K > 64 || !q || I < 1 || I > (1 << 24) || R < 1 || R > K)
        return hipErrorInvalidValue;
    const bool staged = evd_lds_bytes(K, I, true, true) + kStaticLdsMargin <= kLdsLimit;
    if (!staged && !u64) return hipErrorInvalidValue;
    const size_t lds = evd_lds_bytes(K, I, true, staged);
    if (lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
    const int Ii = static_cast<int>(I);
    if (dbl)
        return launch_evd_tri<double, true>(c, K, nullptr, nullptr, flags,
                                            static_cast<const double*>(q), Ii, R, use_v,
                                            static_cast<double*>(u_out),
                                            static_cast<double*>(m_out), sigma, u64,
                                            staged ? 1 : 0, lds, s);
    return launch_evd_tri<float, true>(c, K, nullptr, nullptr, flags, static_cast<const float*>(q),
                                       Ii, R, use_v, static_cast<float*>(u_out),
                                       static_cast<float*>(m_out), sigma, u64, staged ? 1 : 0,
                                       lds, s);
}

hipError_t launch_evd(const double* c, int K, double* v, double* lambda, uint32_t* flags,
                      hipStream_t s) {
    if (K < 1 || K > 64) return hipErrorInvalidValue;
    const size_t lds = evd_lds_bytes(K, 0, false, false);
    if (lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
    return launch_evd_tri<double, false>(c, K, v, lambda, flags, nullptr, 0, 0, 0, nullptr,
                                         nullptr, nullptr, nullptr, 0, lds, s);
}

// Batched QR (all jobs Householder-eligible: I <= 256, K <= 64) and batched
// EVD + factor step; `ns` / `kb` select the template every job of the launch
// shares, `lds` the largest dynamic LDS among them.
hipError_t launch_hqr_batch(const QrJob* jobs, int njobs, int ns, size_t lds, hipStream_t s) {
    if (njobs < 1 || lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
    switch (ns) {
        case 1: hipLaunchKernelGGL((k_hqr_batch<1, 16>), dim3(njobs), dim3(kBlock), lds, s, jobs); break;
        case 2: hipLaunchKernelGGL((k_hqr_batch<2, 16>), dim3(njobs), dim3(kBlock), lds, s, jobs); break;
        case 3: hipLaunchKernelGGL((k_hqr_batch<3, 16>), dim3(njobs), dim3(kBlock), lds, s, jobs); break;
        case 4: hipLaunchKernelGGL((k_hqr_batch<4, 16>), dim3(njobs), dim3(kBlock), lds, s, jobs); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t hqr_lds_bytes(int I, int K) {
    (void)I;
    return static_cast<size_t>(K) * 16 * 16 * sizeof(double);
}

bool evd_factor_staged(int K, int64_t I) {
    return evd_lds_bytes(K, I, true, true) + kStaticLdsMargin <= kLdsLimit;
}

size_t evd_factor_lds_bytes(int K, int64_t I, bool staged) { return evd_lds_bytes(K, I, true, staged); }

hipError_t launch_evd_factor_batch(bool dbl, const EvdJob* jobs, int njobs, int kb, size_t lds,
                                   hipStream_t s) {
    if (njobs < 1 || lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
#define RH_EVB_CASE(KBV)                                                                           \
    case KBV:                                                                                      \
        if (dbl)                                                                                   \
            hipLaunchKernelGGL((k_evd_factor_batch<KBV, double>), dim3(njobs), dim3(kBlock), lds, \
                               s, jobs);                                                           \
        else                                                                                       \
            hipLaunchKernelGGL((k_evd_factor_batch<KBV, float>), dim3(njobs), dim3(kBlock), lds,  \
                               s, jobs);                                                           \
        break;
    switch (kb) {
        RH_EVB_CASE(8)
        RH_EVB_CASE(16)
        RH_EVB_CASE(24)
        RH_EVB_CASE(32)
        RH_EVB_CASE(40)
        RH_EVB_CASE(48)
        RH_EVB_CASE(56)
        RH_EVB_CASE(64)
        default:
            return hipErrorInvalidValue;
    }
#undef RH_EVB_CASE
    return hipGetLastError();
}

}  // namespace rh
