// Small dense steps between the streaming passes, written for latency:
//   k_reduce_parts  fixed-order sum of per-workgroup partials (many workgroups)
//   k_cqr_lds       CholeskyQR2 of Y (I x K) with Y resident in LDS; the K x K
//                   Cholesky factor and its inverse are computed by one wave
//                   without workgroup barriers (Algorithm 1 step 3)
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
// CholeskyQR2 with W = Y resident in LDS (row-major, pitch KP = K | 1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_wave_barrier();
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

// G (column-major K x K, full) = W^T W + shift I; 2x2 register blocks over
// the upper triangle, one block per thread.
__device__ void lds_gram(const double* W, int I, int K, int KP, double* G, double shift) {
    const int KH = (K + 1) / 2;
    const int nblk = KH * (KH + 1) / 2;
    for (int bidx = threadIdx.x; bidx < nblk; bidx += kBlock) {
        // unrank (A, B) with A <= B
        int A = 0, rem = bidx;
        while (rem >= KH - A) {
            rem -= KH - A;
            ++A;
        }
        const int B = A + rem;
        const int a0 = 2 * A, b0 = 2 * B;
        const bool a1ok = a0 + 1 < K, b1ok = b0 + 1 < K;
        double s00 = 0, s01 = 0, s10 = 0, s11 = 0;
        for (int i = 0; i < I; ++i) {
            const double* row = W + i * KP;
            const double x0 = row[a0], x1 = a1ok ? row[a0 + 1] : 0.0;
            const double y0 = row[b0], y1 = b1ok ? row[b0 + 1] : 0.0;
            s00 = fma(x0, y0, s00);
            s01 = fma(x0, y1, s01);
            s10 = fma(x1, y0, s10);
            s11 = fma(x1, y1, s11);
        }
        const double v[2][2] = {{s00, s01}, {s10, s11}};
        for (int da = 0; da < 2; ++da)
            for (int db = 0; db < 2; ++db) {
                const int a = a0 + da, b = b0 + db;
                if (a < K && b < K && a <= b) {
                    const double x = v[da][db] + (a == b ? shift : 0.0);
                    G[b * K + a] = x;
                    G[a * K + b] = x;
                }
            }
    }
    __syncthreads();
}

// One wave: in-place lower Cholesky of G (column-major), then Li = L^{-1}
// (lower, column-major).  Returns false (uniformly) on a pivot below
// 1e-14 of its original diagonal.
__device__ bool wave_chol_inv(double* G, double* Li, int K) {
    const int lane = threadIdx.x & 63;
    bool ok = true;
    for (int j = 0; j < K; ++j) {
        double s = 0.0;
        if (lane >= j && lane < K) {
            s = G[j * K + lane];
            for (int m = 0; m < j; ++m) s -= G[m * K + lane] * G[m * K + j];
        }
        const double d = __shfl(s, j, kWave);
        const double d0 = G[j * K + j];          // not yet overwritten
        if (!(d > 1e-14 * d0) || !(d0 > 0.0)) {
            ok = false;
            break;
        }
        const double r = sqrt(d);
        if (lane == j) G[j * K + j] = r;
        if (lane > j && lane < K) G[j * K + lane] = s / r;
        wave_sync_lds();
    }
    if (!ok) return false;
    // column c = lane of L^{-1}: forward substitution, own column only
    const int c = lane;
    if (c < K) {
        for (int i = 0; i < K; ++i) {
            double x = 0.0;
            if (i >= c) {
                double s = (i == c) ? 1.0 : 0.0;
                for (int m = c; m < i; ++m) s -= G[m * K + i] * Li[m * K + c];
                x = s / G[i * K + i];
            }
            Li[i * K + c] = x;     // Li(i, c) stored row-major: Li[i * K + c]
        }
    }
    wave_sync_lds();
    return true;
}

// W2 = W L^{-T}: W2(i, j) = sum_{m <= j} W(i, m) Linv(j, m); lanes over rows,
// blocks of 4 output columns per item.
__device__ void lds_apply(const double* W, double* W2, int I, int K, int KP, const double* Li) {
    const int JB = (K + 3) / 4;
    for (int item = threadIdx.x; item < I * JB; item += kBlock) {
        const int jb = item / I, i = item - jb * I;
        const int j0 = 4 * jb;
        const double* row = W + i * KP;
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        const int mmax = (j0 + 3 < K - 1) ? j0 + 3 : K - 1;
        for (int m = 0; m <= mmax; ++m) {
            const double w = row[m];
            s0 = fma(w, (j0 + 0 < K) ? Li[(j0 + 0) * K + m] : 0.0, s0);
            s1 = fma(w, (j0 + 1 < K) ? Li[(j0 + 1) * K + m] : 0.0, s1);
            s2 = fma(w, (j0 + 2 < K) ? Li[(j0 + 2) * K + m] : 0.0, s2);
            s3 = fma(w, (j0 + 3 < K) ? Li[(j0 + 3) * K + m] : 0.0, s3);
        }
        double* o = W2 + i * KP;
        if (j0 + 0 < K) o[j0 + 0] = s0;
        if (j0 + 1 < K) o[j0 + 1] = s1;
        if (j0 + 2 < K) o[j0 + 2] = s2;
        if (j0 + 3 < K) o[j0 + 3] = s3;
    }
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cqr_lds(const double* __restrict__ y, int I, int K,
                                                    double* work, double* q64, T* q_out,
                                                    uint32_t* flags) {
    extern __shared__ __align__(16) double shd[];
    const int KP = K | 1;
    double* W = shd;
    double* W2 = W + I * KP;
    double* G = W2 + I * KP;
    double* Li = G + K * K;
    __shared__ double tau_s[RHOSVD_MAX_K], alpha_s[RHOSVD_MAX_K];
    __shared__ double red[kBlock / kWave];
    __shared__ int ok_sh;
    const int tid = threadIdx.x;
    for (int e = tid; e < I * K; e += kBlock) {
        const int k = e / I, i = e - k * I;
        W[i * KP + k] = y[e];
    }
    __syncthreads();
    lds_gram(W, I, K, KP, G, 0.0);
    bool shifted = false;
    if (tid < kWave) {
        const bool ok = wave_chol_inv(G, Li, K);
        if (tid == 0) ok_sh = ok;
    }
    __syncthreads();
    if (!ok_sh) {
        // shifted CholeskyQR (Fukaya et al., SISC 2020): G + s I with
        // s = 11 (I K + K (K + 1)) u ||Y||_F^2
        shifted = true;
        double tr = 0.0;
        for (int e = tid; e < I * K; e += kBlock) {
            const double v = y[e];
            tr += v * v;
        }
        tr = wave_sum(tr);
        if ((tid & 63) == 0) red[tid >> 6] = tr;
        __syncthreads();
        const double trace = red[0] + red[1] + red[2] + red[3];
        const double shift = 11.0 * (static_cast<double>(I) * K + static_cast<double>(K) * (K + 1)) *
                             1.1102230246251565e-16 * trace;
        lds_gram(W, I, K, KP, G, shift);
        if (tid < kWave) {
            const bool ok = wave_chol_inv(G, Li, K);
            if (tid == 0) ok_sh = ok;
        }
        __syncthreads();
    }
    bool ok = ok_sh;
    const int rounds = shifted ? 3 : 2;
    double* cur = W;
    double* nxt = W2;
    for (int r = 0; r < rounds && ok; ++r) {
        if (r > 0) {
            lds_gram(cur, I, K, KP, G, 0.0);
            if (tid < kWave) {
                const bool okw = wave_chol_inv(G, Li, K);
                if (tid == 0) ok_sh = okw;
            }
            __syncthreads();
            ok = ok_sh;
            if (!ok) break;
        }
        lds_apply(cur, nxt, I, K, KP, Li);
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    if (ok) {
        for (int e = tid; e < I * K; e += kBlock) {
            const int k = e / I, i = e - k * I;
            const double v = cur[i * KP + k];
            q64[e] = v;
            q_out[e] = static_cast<T>(v);
        }
    } else {
        householder_qr(y, I, K, work, q64, tau_s, alpha_s, red);
        for (int e = tid; e < I * K; e += kBlock) q_out[e] = static_cast<T>(q64[e]);
    }
    if (tid == 0 && flags) {
        uint32_t f = shifted ? RHOSVD_FLAG_CQR_SHIFTED : 0u;
        if (!ok) f |= RHOSVD_FLAG_QR_HOUSEHOLDER;
        if (f) atomicOr(flags, f);
    }
}

size_t cqr_lds_bytes(int64_t I, int K) {
    const int KP = K | 1;
    return (2 * static_cast<size_t>(I) * KP + 2 * static_cast<size_t>(K) * K) * sizeof(double);
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
    if (cqr_lds_bytes(I, K) + kStaticLdsMargin > kLdsLimit)
        return launch_cqr_global(y, I, K, dbl, q_out, q64, flags, s);
    return launch_cqr_lds(y, I, K, dbl, q_out, q64, flags, s);
}

hipError_t launch_cqr_lds(const double* y, int64_t I, int K, bool dbl, void* q_out, double* q64,
                          uint32_t* flags, hipStream_t s) {
    double* work = q64 + I * K;
    const size_t lds = cqr_lds_bytes(I, K);
    if (lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
    if (dbl)
        hipLaunchKernelGGL(k_cqr_lds<double>, dim3(1), dim3(kBlock), lds, s, y,
                           static_cast<int>(I), K, work, q64, static_cast<double*>(q_out), flags);
    else
        hipLaunchKernelGGL(k_cqr_lds<float>, dim3(1), dim3(kBlock), lds, s, y, static_cast<int>(I),
                           K, work, q64, static_cast<float*>(q_out), flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Jacobi EVD (cyclic, round-robin parallel ordering, rotations as in Golub &
// Van Loan sym.schur2) of A (LDS, row-major Ke x Ke, Ke <= 64) accumulating
// V.  A round applies its Ke/2 disjoint rotations J at once: with, for every
// index i, alpha_i = c and beta_i = -s (i the first of its pair) or +s (the
// second), and partner p(i),
//   A'(i,j) = a_i (a_j A(i,j) + b_j A(i,p(j))) + b_i (a_j A(p(i),j) + b_j A(p(i),p(j)))
//   V'(i,j) = a_j V(i,j) + b_j V(i,p(j))
// computed from the old A into a second buffer (two barriers per round).
// Stops when the off-diagonal mass is below 1e-28 of the total (relative RMS
// 1e-14); rotations with |a_pq| <= 1e-18 sqrt|a_pp a_qq| are skipped, and a
// round whose rotations are all skipped costs one barrier.
// ---------------------------------------------------------------------------
constexpr int kSweeps = 30;

__device__ bool jacobi_lds(double*& A, double*& A2, double*& V, double*& V2, int Ke, int* sweeps) {
    // rotation data is double-buffered by round parity: a wave can run at
    // most one round ahead of another (every round has a barrier after its
    // rotation step), so it never overwrites what a slower wave still reads
    __shared__ double alpha[2][RHOSVD_MAX_K], beta[2][RHOSVD_MAX_K];
    __shared__ int partner[2][RHOSVD_MAX_K];
    __shared__ int rot[2][RHOSVD_MAX_K / 2];
    __shared__ double red[2][kBlock / kWave];
    __shared__ int conv;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = Ke / 2;
    const int n1 = Ke - 1;
    for (int sweep = 0; sweep < kSweeps; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int r = wave; r < Ke; r += kBlock / kWave) {
            if (lane < Ke) {
                const double v = A[r * Ke + lane] * A[r * Ke + lane];
                tot += v;
                if (r != lane) off += v;
            }
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
            const int b = round & 1;
            if (tid < half) {
                const int m = tid;
                int x0 = m - 1 + round;
                if (x0 >= n1) x0 -= n1;
                int x1 = Ke - 2 - m + round;
                if (x1 >= n1) x1 -= n1;
                const int a0 = (m == 0) ? 0 : 1 + x0;
                const int a1 = 1 + x1;
                const int p = a0 < a1 ? a0 : a1;
                const int q = a0 < a1 ? a1 : a0;
                const double apq = A[p * Ke + q];
                const double app = A[p * Ke + p], aqq = A[q * Ke + q];
                double c = 1.0, s = 0.0;
                int r = 0;
                if (apq != 0.0 && fabs(apq) > 1e-18 * sqrt(fabs(app * aqq))) {
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                    r = 1;
                }
                alpha[b][p] = c;
                beta[b][p] = -s;
                partner[b][p] = q;
                alpha[b][q] = c;
                beta[b][q] = s;
                partner[b][q] = p;
                rot[b][m] = r;
            }
            __syncthreads();
            int any = 0;
            for (int m = 0; m < half; ++m) any |= rot[b][m];
            if (!any) continue;
            for (int i = wave; i < Ke; i += kBlock / kWave) {
                if (lane < Ke) {
                    const int j = lane;
                    const int pi = partner[b][i], pj = partner[b][j];
                    const double ai = alpha[b][i], bi = beta[b][i], aj = alpha[b][j], bj = beta[b][j];
                    const double x = aj * A[i * Ke + j] + bj * A[i * Ke + pj];
                    const double y = aj * A[pi * Ke + j] + bj * A[pi * Ke + pj];
                    A2[i * Ke + j] = ai * x + bi * y;
                    V2[i * Ke + j] = aj * V[i * Ke + j] + bj * V[i * Ke + pj];
                }
            }
            __syncthreads();
            double* t = A;
            A = A2;
            A2 = t;
            t = V;
            V = V2;
            V2 = t;
        }
    }
    return false;
}

// EVD of C (K x K, column-major, device) and, when q != nullptr, the factor
// step: U = Q V[:, :R] (V = identity when use_v == 0), canonical signs, M =
// V_R diag(s) (K x R), sigma = sqrt(max(lambda, 0))[:R].  The sorted
// eigenpairs also go to v_out / lam_out when those are non-null.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_evd_factor(const double* __restrict__ cin, int K,
                                                       double* v_out, double* lam_out,
                                                       uint32_t* flags, const T* __restrict__ q,
                                                       int I, int R, int use_v,
                                                       T* __restrict__ u_out,
                                                       T* __restrict__ m_out,
                                                       double* __restrict__ sigma,
                                                       double* __restrict__ u64) {
    extern __shared__ __align__(16) double shd[];
    const int Ke = K + (K & 1);
    double* A = shd;
    double* V = A + Ke * Ke;
    double* A2 = V + Ke * Ke;
    double* V2 = A2 + Ke * Ke;
    __shared__ double lam[RHOSVD_MAX_K];
    __shared__ double sgn[RHOSVD_MAX_K];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < Ke * Ke; e += kBlock) {
        const int r = e / Ke, c = e - r * Ke;
        A[e] = (r < K && c < K) ? cin[c * K + r] : 0.0;
        V[e] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    int sweeps = 0;
    const bool conv = jacobi_lds(A, A2, V, V2, Ke, &sweeps);
    if (tid == 0 && !conv && flags) atomicOr(flags, RHOSVD_FLAG_EVD_NOCONV);
    // the stand-alone EVD reports its sweep count in bits 16..23 of flags
    if (tid == 0 && flags && !q) atomicOr(flags, static_cast<uint32_t>(sweeps & 0xff) << 16);
    double* Vs = A2;                   // sorted eigenvectors (K x K, column-major) in the free buffer
    for (int i = tid; i < K; i += kBlock) {
        const double li = A[i * Ke + i];
        int rank = 0;
        for (int j = 0; j < K; ++j) {
            const double lj = A[j * Ke + j];
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
    // U = Q V_R (FP64), canonical signs
    for (int e = tid; e < I * R; e += kBlock) {
        const int r = e / I, i = e - r * I;
        double s = 0.0;
        if (use_v) {
            for (int k = 0; k < K; ++k)
                s += static_cast<double>(q[static_cast<int64_t>(k) * I + i]) * Vs[r * K + k];
        } else {
            s = static_cast<double>(q[static_cast<int64_t>(r) * I + i]);
        }
        u64[e] = s;
    }
    __syncthreads();
    for (int r = wave; r < R; r += kBlock / kWave) {
        double best = -1.0;
        int bi = 0x7fffffff;
        for (int i = lane; i < I; i += kWave) {
            const double a = fabs(u64[static_cast<int64_t>(r) * I + i]);
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
        if (lane == 0) sgn[r] = (u64[static_cast<int64_t>(r) * I + bi] < 0.0) ? -1.0 : 1.0;
    }
    __syncthreads();
    for (int e = tid; e < I * R; e += kBlock) u_out[e] = static_cast<T>(sgn[e / I] * u64[e]);
    for (int e = tid; e < K * R; e += kBlock) {
        const int r = e / K, k = e - r * K;
        const double vv = use_v ? Vs[r * K + k] : (k == r ? 1.0 : 0.0);
        m_out[e] = static_cast<T>(sgn[r] * vv);
    }
    if (sigma)
        for (int r = tid; r < R; r += kBlock) sigma[r] = sqrt(fmax(lam[r], 0.0));
}

hipError_t launch_evd(const double* c, int K, double* v, double* lambda, uint32_t* flags,
                      hipStream_t s);

size_t evd_lds_bytes(int K) {
    const int Ke = K + (K & 1);
    return 4 * static_cast<size_t>(Ke) * Ke * sizeof(double);
}

hipError_t launch_evd_factor(bool dbl, const double* c, int K, double* v_out, double* lam_out,
                             uint32_t* flags, const void* q, int64_t I, int R, int use_v,
                             void* u_out, void* m_out, double* sigma, double* u64, hipStream_t s) {
    const size_t lds = evd_lds_bytes(K);
    if (K < 1 || K > 64 || lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
    if (dbl)
        hipLaunchKernelGGL(k_evd_factor<double>, dim3(1), dim3(kBlock), lds, s, c, K, v_out,
                           lam_out, flags, static_cast<const double*>(q), static_cast<int>(I), R,
                           use_v, static_cast<double*>(u_out), static_cast<double*>(m_out), sigma,
                           u64);
    else
        hipLaunchKernelGGL(k_evd_factor<float>, dim3(1), dim3(kBlock), lds, s, c, K, v_out,
                           lam_out, flags, static_cast<const float*>(q), static_cast<int>(I), R,
                           use_v, static_cast<float*>(u_out), static_cast<float*>(m_out), sigma,
                           u64);
    return hipGetLastError();
}

}  // namespace rh

namespace rh {
hipError_t launch_evd(const double* c, int K, double* v, double* lambda, uint32_t* flags,
                      hipStream_t s) {
    return launch_evd_factor(true, c, K, v, lambda, flags, nullptr, 0, 0, 0, nullptr, nullptr,
                             nullptr, nullptr, s);
}
}  // namespace rh
