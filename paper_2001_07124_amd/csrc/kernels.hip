// HIP kernels of the randomized HOSVD hot path for gfx950.
//
// Streaming passes (one read of the current tensor each):
//   OP_SKETCH  Y = S_(n) Omega          Algorithm 1 step 2 (q = 0) / Algorithm 6 step 3
//   OP_POWER   Y = S_(n) (S_(n)^T Q)    Algorithm 1 step 2, one power step, fused
//   OP_TTM     out = S x_n M^T (+ Gram) Algorithm 1 step 4 (B = Q^T S_(n)) and the
//                                       truncation S x_n U^T of Algorithm 8 step 4
// Small single-workgroup kernels: CholeskyQR2 (step 3), Jacobi EVD (step 5),
// factor + sign canonicalisation (steps 6-7), fixed-order reductions.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "householder.hpp"
#include "kernels.hpp"
#include "rhosvd.h"

namespace rh {

constexpr int kMaxT1 = 16;   // Y accumulator tiles (16x16) per wave
constexpr int kMaxT2 = 8;    // Z tiles per wave
constexpr int kMaxTG = 16;   // Gram tiles per wave
constexpr size_t kStreamLdsCap = 80 * 1024;

// ---------------------------------------------------------------------------
// Streaming contraction over an n-unfolding view (L, I, T).
// A workgroup walks tiles of C unfolding columns (grid-stride).  Each tile
// S[:, j0:j0+C) is staged in LDS as sS[c][i] (pitch P), zero-padded to
// I_pad rows.  The K-wide right operand (Omega tile or Z = S^T Q) sits in
// sW[c][k] (pitch KW); Q / M sits in sQ[i][k].
// ---------------------------------------------------------------------------
// The body walks the tiles t_begin, t_begin + t_step, ... < g.ntiles and
// writes its partials into slot `gidx` of a.part_y / a.part_g / a.part_ss.
template <typename T, int OP>
__device__ __forceinline__ void stream_body(const StreamGeom& g, const StreamArgs& a, int want_ss,
                                            int want_gram, int64_t t_begin, int64_t t_step,
                                            size_t gidx) {
    using MM = Mma<T>;
    using acc_t = typename MM::acc_t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sS = reinterpret_cast<T*>(smem_raw);
    T* sW = sS + g.C * g.P;
    T* sQ = sW + g.C * g.KW;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lane16 = lane & 15, quad = lane >> 4;
    const T* __restrict__ src = static_cast<const T*>(a.src);
    const int I = static_cast<int>(g.I), K = g.K, C = g.C, P = g.P, KW = g.KW;
    const int NB = g.K_pad / 16, CB = C / 16;
    const int64_t L = g.L, J = g.J;

    const int lds_elems = C * P + C * KW + (OP != OP_SKETCH ? g.I_pad * KW : 0);
    for (int e = tid; e < lds_elems; e += kBlock) sS[e] = T(0);
    __syncthreads();
    if (OP != OP_SKETCH) {
        const T* __restrict__ m = static_cast<const T*>(a.mat);
        for (int e = tid; e < I * K; e += kBlock) {
            const int k = e / I, i = e - k * I;
            sQ[i * KW + k] = m ? m[e] : T(i == k ? 1 : 0);
        }
    }
    __syncthreads();

    acc_t acc1[kMaxT1];
    acc_t accg[kMaxTG];
#pragma unroll
    for (int m = 0; m < kMaxT1; ++m) acc1[m] = zero4<acc_t>();
#pragma unroll
    for (int m = 0; m < kMaxTG; ++m) accg[m] = zero4<acc_t>();
    double ss = 0.0;
    const int np1 = (g.I_pad / 16) * NB;
    const int np2 = CB * NB;
    const int npg = NB * NB;

    for (int64_t tile = t_begin; tile < g.ntiles; tile += t_step) {
        const int64_t j0 = tile * C;
        const int Cv = static_cast<int>(J - j0 < C ? J - j0 : C);

        // ---- stage the tile S[:, j0 : j0 + Cv) into sS[c][i]
        if (L == 1) {
            const T* __restrict__ base = src + j0 * static_cast<int64_t>(I);
            const int n = Cv * I;
            for (int e = tid; e < n; e += kBlock) {
                const int c = e / I, i = e - c * I;
                const T v = base[e];
                sS[c * P + i] = v;
                if (want_ss) ss += static_cast<double>(v) * static_cast<double>(v);
            }
        } else {
            const int c = tid % C;
            if (c < Cv) {
                const int64_t j = j0 + c;
                const int64_t t = j / L;
                const int64_t l = j - t * L;
                const T* __restrict__ colp = src + l + L * static_cast<int64_t>(I) * t;
                for (int i = tid / C; i < I; i += kBlock / C) {
                    const T v = colp[L * i];
                    sS[c * P + i] = v;
                    if (want_ss) ss += static_cast<double>(v) * static_cast<double>(v);
                }
            }
        }
        if (Cv < C) {
            for (int e = tid; e < (C - Cv) * I; e += kBlock) {
                const int c = Cv + e / I, i = e % I;
                sS[c * P + i] = T(0);
            }
        }

        // ---- Omega tile: entries (j0 + c, k) for c < Cv, k < K
        if (OP == OP_SKETCH && (g.L > 1 || a.kr.nq)) {
            // generator rows are not consecutive along the tile's columns
            // (or the structured matrix): entry by entry
            for (int it = tid; it < K * Cv; it += kBlock) {
                const int k = it / Cv, c = it - k * Cv;
                sW[c * KW + k] = a.kr.nq ? kr_entry<T>(a.kr, j0 + c, k)
                                         : omega_entry<T>(a.seed, a.mode, a.tag, j0 + c, k, g.L, g.T, J);
            }
        } else if (OP == OP_SKETCH) {
            const int QPK = C / 4 + 2;
            for (int it = tid; it < K * QPK; it += kBlock) {
                const int k = it / QPK, qi = it - k * QPK;
                const uint64_t e_lo = static_cast<uint64_t>(k) * static_cast<uint64_t>(J) +
                                      static_cast<uint64_t>(j0);
                const uint64_t e_hi = e_lo + static_cast<uint64_t>(Cv);
                const uint64_t q = (e_lo >> 2) + static_cast<uint64_t>(qi);
                if (4 * q >= e_hi) continue;
                T z[4];
                normals4<T>(q, a.mode, a.tag, a.seed, z);
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const uint64_t e = 4 * q + w;
                    if (e >= e_lo && e < e_hi) sW[static_cast<int>(e - e_lo) * KW + k] = z[w];
                }
            }
            if (Cv < C) {
                for (int e = tid; e < (C - Cv) * K; e += kBlock) {
                    const int c = Cv + e / K, k = e % K;
                    sW[c * KW + k] = T(0);
                }
            }
        }
        __syncthreads();

        // ---- Z = S_tile^T Q  (C x K_pad), into sW
        if (OP == OP_POWER || OP == OP_TTM) {
            acc_t acc2[kMaxT2];
#pragma unroll
            for (int m = 0; m < kMaxT2; ++m) acc2[m] = zero4<acc_t>();
            for (int ks = 0; ks < g.I_pad / 4; ++ks) {
                const int kr = ks * 4 + quad;
#pragma unroll
                for (int m = 0; m < kMaxT2; ++m) {
                    const int p = wave + 4 * m;
                    if (p < np2) {
                        const int cb = p / NB, nb = p - cb * NB;
                        const T av = sS[(cb * 16 + lane16) * P + kr];
                        const T bv = sQ[kr * KW + nb * 16 + lane16];
                        acc2[m] = MM::step(av, bv, acc2[m]);
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < kMaxT2; ++m) {
                const int p = wave + 4 * m;
                if (p < np2) {
                    const int cb = p / NB, nb = p - cb * NB;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        sW[(cb * 16 + MM::row(quad, r)) * KW + nb * 16 + lane16] = acc2[m][r];
                }
            }
            __syncthreads();
        }

        // ---- Y += S_tile W   (I_pad x K_pad)
        if (OP == OP_SKETCH || OP == OP_POWER) {
            for (int ks = 0; ks < C / 4; ++ks) {
                const int kr = ks * 4 + quad;
#pragma unroll
                for (int m = 0; m < kMaxT1; ++m) {
                    const int p = wave + 4 * m;
                    if (p < np1) {
                        const int ib = p / NB, nb = p - ib * NB;
                        const T av = sS[kr * P + ib * 16 + lane16];
                        const T bv = sW[kr * KW + nb * 16 + lane16];
                        acc1[m] = MM::step(av, bv, acc1[m]);
                    }
                }
            }
        }

        // ---- write the folded output and accumulate its Gram
        if (OP == OP_TTM) {
            T* __restrict__ out = static_cast<T*>(a.out);
            if (L == 1 && a.out_t) {
                for (int e = tid; e < Cv * K; e += kBlock) {
                    const int k = e / Cv, c = e - k * Cv;
                    out[static_cast<int64_t>(k) * J + j0 + c] = sW[c * KW + k];
                }
            } else if (L == 1) {
                T* __restrict__ ob = out + j0 * static_cast<int64_t>(K);
                for (int e = tid; e < Cv * K; e += kBlock) {
                    const int c = e / K, k = e - c * K;
                    ob[e] = sW[c * KW + k];
                }
            } else {
                const int c = tid % C;
                if (c < Cv) {
                    const int64_t j = j0 + c;
                    const int64_t t = j / L;
                    const int64_t l = j - t * L;
                    T* __restrict__ op = out + l + L * static_cast<int64_t>(K) * t;
                    for (int k = tid / C; k < K; k += kBlock / C) op[L * k] = sW[c * KW + k];
                }
            }
            if (want_gram) {
                for (int ks = 0; ks < C / 4; ++ks) {
                    const int kr = ks * 4 + quad;
#pragma unroll
                    for (int m = 0; m < kMaxTG; ++m) {
                        const int p = wave + 4 * m;
                        if (p < npg) {
                            const int kb = p / NB, kb2 = p - kb * NB;
                            const T av = sW[kr * KW + kb * 16 + lane16];
                            const T bv = sW[kr * KW + kb2 * 16 + lane16];
                            accg[m] = MM::step(av, bv, accg[m]);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }

    // ---- per-workgroup partials
    if (OP == OP_SKETCH || OP == OP_POWER) {
        T* __restrict__ py = static_cast<T*>(a.part_y) + gidx * g.K_pad * g.I_pad;
#pragma unroll
        for (int m = 0; m < kMaxT1; ++m) {
            const int p = wave + 4 * m;
            if (p < np1) {
                const int ib = p / NB, nb = p - ib * NB;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    py[(nb * 16 + lane16) * g.I_pad + ib * 16 + MM::row(quad, r)] = acc1[m][r];
            }
        }
    }
    if (OP == OP_TTM && want_gram) {
        T* __restrict__ pg = static_cast<T*>(a.part_g) + gidx * g.K_pad * g.K_pad;
#pragma unroll
        for (int m = 0; m < kMaxTG; ++m) {
            const int p = wave + 4 * m;
            if (p < npg) {
                const int kb = p / NB, kb2 = p - kb * NB;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    pg[(kb2 * 16 + lane16) * g.K_pad + kb * 16 + MM::row(quad, r)] = accg[m][r];
            }
        }
    }
    if (want_ss) {
        __shared__ double red[kBlock / kWave];
        ss = wave_sum(ss);
        if (lane == 0) red[wave] = ss;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w) s += red[w];
            a.part_ss[gidx] = s;
        }
    }
}

template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_stream(StreamGeom g, StreamArgs a, int want_ss,
                                                   int want_gram) {
    stream_body<T, OP>(g, a, want_ss, want_gram, blockIdx.x, gridDim.x, blockIdx.x);
}

// Many independent passes in one launch: workgroup (x, y) serves job y as
// its workgroup x of jobs[y].units (the others return at once), with the
// job's own geometry and buffers.
template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_stream_batch(const StreamJob* __restrict__ jobs) {
    const StreamJob& jb = jobs[blockIdx.y];
    if (static_cast<int>(blockIdx.x) >= jb.units) return;
    const StreamGeom g = jb.g;
    const StreamArgs a = jb.a;
    stream_body<T, OP>(g, a, a.part_ss != nullptr, a.part_g != nullptr, blockIdx.x, jb.units,
                       blockIdx.x);
}

static int round16(int64_t v) { return static_cast<int>((v + 15) / 16 * 16); }

bool plan_stream(int op, int elem, int64_t L, int64_t I, int64_t T, int K, int num_cu,
                 StreamGeom* g, int cmax) {
    if (L < 1 || I < 1 || T < 1 || K < 1 || K > RHOSVD_MAX_K) return false;
    if (I > 4096) return false;
    g->L = L;
    g->I = I;
    g->T = T;
    g->J = L * T;
    g->K = K;
    g->I_pad = round16(I);
    g->K_pad = round16(K);
    const int NB = g->K_pad / 16, IB = g->I_pad / 16;
    if ((op == OP_SKETCH || op == OP_POWER) && IB * NB > 4 * kMaxT1) return false;
    if (op == OP_TTM && NB * NB > 4 * kMaxTG) return false;
    // pitches: rows of 16 consecutive values read by four lane groups
    // land in disjoint bank ranges when the pitch is 16 or 48 mod 64 words
    g->KW = g->K_pad + ((g->K_pad % 32 == 0) ? 16 : 0);
    g->P = (op == OP_SKETCH) ? g->I_pad + ((g->I_pad % 32 == 0) ? 16 : 0) : g->I_pad + 1;
    // the widest column tile within kStreamLdsCap (two workgroups per CU);
    // when none fits (tall modes, whose staged M alone takes most of it), the
    // widest within the whole LDS
    const int cands[3] = {64, 32, 16};
    const size_t caps[2] = {kStreamLdsCap, kLdsLimit - kStaticLdsMargin};
    g->C = 0;
    for (int pass = 0; pass < 2 && g->C == 0; ++pass) {
        for (int ci = 0; ci < 3; ++ci) {
            const int C = cands[ci];
            if (C > cmax) continue;
            if ((op == OP_POWER || op == OP_TTM) && (C / 16) * NB > 4 * kMaxT2) continue;
            size_t elems = static_cast<size_t>(C) * g->P + static_cast<size_t>(C) * g->KW;
            if (op != OP_SKETCH) elems += static_cast<size_t>(g->I_pad) * g->KW;
            if (elems * elem <= caps[pass]) {
                g->C = C;
                g->lds_bytes = elems * elem;
                break;
            }
        }
    }
    if (g->C == 0) return false;
    g->ntiles = (g->J + g->C - 1) / g->C;
    const int64_t cap = static_cast<int64_t>(num_cu > 0 ? num_cu : 256) * 2;
    g->grid = static_cast<int>(g->ntiles < cap ? g->ntiles : cap);
    return true;
}

template <typename T, int OP>
static hipError_t launch_stream_t(const StreamGeom& g, const StreamArgs& a, hipStream_t s) {
    const int want_ss = a.part_ss != nullptr;
    const int want_gram = a.part_g != nullptr;
    hipLaunchKernelGGL((k_stream<T, OP>), dim3(g.grid), dim3(kBlock), g.lds_bytes, s, g, a,
                       want_ss, want_gram);
    return hipGetLastError();
}

hipError_t launch_stream(int op, bool dbl, const StreamGeom& g, const StreamArgs& a,
                         hipStream_t s) {
    if (dbl) {
        if (op == OP_SKETCH) return launch_stream_t<double, OP_SKETCH>(g, a, s);
        if (op == OP_POWER) return launch_stream_t<double, OP_POWER>(g, a, s);
        return launch_stream_t<double, OP_TTM>(g, a, s);
    }
    if (op == OP_SKETCH) return launch_stream_t<float, OP_SKETCH>(g, a, s);
    if (op == OP_POWER) return launch_stream_t<float, OP_POWER>(g, a, s);
    return launch_stream_t<float, OP_TTM>(g, a, s);
}

template <typename T, int OP>
static hipError_t launch_stream_batch_t(const StreamJob* jobs, int njobs, int max_units,
                                        size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_stream_batch<T, OP>), dim3(max_units, njobs), dim3(kBlock), lds, s,
                       jobs);
    return hipGetLastError();
}

hipError_t launch_stream_batch(int op, bool dbl, const StreamJob* jobs, int njobs, int max_units,
                               size_t lds, hipStream_t s) {
    if (njobs < 1 || max_units < 1 || lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
    if (dbl) {
        if (op == OP_SKETCH) return launch_stream_batch_t<double, OP_SKETCH>(jobs, njobs, max_units, lds, s);
        if (op == OP_POWER) return launch_stream_batch_t<double, OP_POWER>(jobs, njobs, max_units, lds, s);
        return launch_stream_batch_t<double, OP_TTM>(jobs, njobs, max_units, lds, s);
    }
    if (op == OP_SKETCH) return launch_stream_batch_t<float, OP_SKETCH>(jobs, njobs, max_units, lds, s);
    if (op == OP_POWER) return launch_stream_batch_t<float, OP_POWER>(jobs, njobs, max_units, lds, s);
    return launch_stream_batch_t<float, OP_TTM>(jobs, njobs, max_units, lds, s);
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of per-workgroup sums of squares.
// ---------------------------------------------------------------------------
__global__ void k_reduce_ss(const double* __restrict__ part, int G, double* __restrict__ out) {
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int i = threadIdx.x; i < G; i += kBlock) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_reduce_ss(const double* part, int G, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_ss, dim3(1), dim3(kBlock), 0, s, part, G, out);
    return hipGetLastError();
}

template <typename T>
__global__ void k_sumsq(const T* __restrict__ x, int64_t n, double* __restrict__ part) {
    __shared__ double red[kBlock / kWave];
    double s = 0.0;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; e < n;
         e += static_cast<int64_t>(gridDim.x) * kBlock) {
        const double v = static_cast<double>(x[e]);
        s += v * v;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) t += red[w];
        part[blockIdx.x] = t;
    }
}

hipError_t launch_sumsq(bool dbl, const void* x, int64_t n, double* part, int G, hipStream_t s) {
    if (dbl)
        hipLaunchKernelGGL(k_sumsq<double>, dim3(G), dim3(kBlock), 0, s,
                           static_cast<const double*>(x), n, part);
    else
        hipLaunchKernelGGL(k_sumsq<float>, dim3(G), dim3(kBlock), 0, s,
                           static_cast<const float*>(x), n, part);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CholeskyQR2 on Y (I x K, FP64).  One workgroup.  Each round forms the Gram
// G = W^T W of the current W in row chunks staged through LDS, factors
// G = L L^T in place (right-looking), inverts L, and writes W L^{-T}.  If the
// first Cholesky meets a pivot below 1e-14 of its original diagonal, the
// round is redone on G + s I with the shift s = 11 (I K + K (K + 1)) u ||Y||_F^2
// (shifted CholeskyQR, Fukaya et al., SISC 2020) and a third round is added.
// ---------------------------------------------------------------------------
constexpr int kCqrRows = 32;

__device__ void cqr_gram(const double* __restrict__ w, int I, int K, double* G, double* ch,
                         double shift) {
    const int tid = threadIdx.x;
    const int CP = kCqrRows + 1;
    double acc[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) acc[m] = 0.0;
    for (int i0 = 0; i0 < I; i0 += kCqrRows) {
        const int rows = (I - i0 < kCqrRows) ? (I - i0) : kCqrRows;
        __syncthreads();
        for (int e = tid; e < rows * K; e += kBlock) {
            const int k = e / rows, r = e - k * rows;
            ch[k * CP + r] = w[static_cast<int64_t>(k) * I + i0 + r];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int e = tid + kBlock * m;
            if (e < K * K) {
                const int a = e % K, b = e / K;
                if (a <= b) {
                    double s = 0.0;
                    for (int r = 0; r < rows; ++r) s += ch[a * CP + r] * ch[b * CP + r];
                    acc[m] += s;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int e = tid + kBlock * m;
        if (e < K * K) {
            const int a = e % K, b = e / K;
            if (a <= b) {
                const double v = acc[m] + (a == b ? shift : 0.0);
                G[b * K + a] = v;
                G[a * K + b] = v;
            }
        }
    }
    __syncthreads();
}

// In-place lower Cholesky of G (column-major); returns true on success.
__device__ bool cqr_cholesky(double* G, int K, double* diag0, int* fail) {
    const int tid = threadIdx.x;
    for (int j = tid; j < K; j += kBlock) diag0[j] = G[j * K + j];
    if (tid == 0) *fail = 0;
    __syncthreads();
    for (int j = 0; j < K; ++j) {
        if (tid == 0) {
            const double d = G[j * K + j];
            if (!(d > 1e-14 * diag0[j]) || !(diag0[j] > 0.0))
                *fail = 1;
            else
                G[j * K + j] = sqrt(d);
        }
        __syncthreads();
        if (*fail) return false;
        const double r = G[j * K + j];
        for (int i = j + 1 + tid; i < K; i += kBlock) G[j * K + i] /= r;
        __syncthreads();
        const int m = K - j - 1;
        for (int e = tid; e < m * m; e += kBlock) {
            const int a = j + 1 + e % m, b = j + 1 + e / m;
            if (a >= b) G[b * K + a] -= G[j * K + a] * G[j * K + b];
        }
        __syncthreads();
    }
    return true;
}

// Linv = L^{-1} (lower), one column per thread by forward substitution.
__device__ void cqr_invert(const double* G, int K, double* Li) {
    const int tid = threadIdx.x;
    for (int e = tid; e < K * K; e += kBlock) Li[e] = 0.0;
    __syncthreads();
    for (int c = tid; c < K; c += kBlock) {
        // solve L x = e_c; x_i = 0 for i < c
        Li[c * K + c] = 1.0 / G[c * K + c];
        for (int i = c + 1; i < K; ++i) {
            double s = 0.0;
            for (int m = c; m < i; ++m) s += G[m * K + i] * Li[c * K + m];
            Li[c * K + i] = -s / G[i * K + i];
        }
    }
    __syncthreads();
}

// dst = src L^{-T}: dst(i, j) = sum_{m <= j} src(i, m) Linv(j, m)
__device__ void cqr_apply(const double* __restrict__ src, int I, int K, const double* Li,
                          double* ch, double* __restrict__ dst) {
    const int tid = threadIdx.x;
    const int CP = kCqrRows + 1;
    for (int i0 = 0; i0 < I; i0 += kCqrRows) {
        const int rows = (I - i0 < kCqrRows) ? (I - i0) : kCqrRows;
        __syncthreads();
        for (int e = tid; e < rows * K; e += kBlock) {
            const int k = e / rows, r = e - k * rows;
            ch[k * CP + r] = src[static_cast<int64_t>(k) * I + i0 + r];
        }
        __syncthreads();
        for (int e = tid; e < rows * K; e += kBlock) {
            const int j = e / rows, r = e - j * rows;
            double s = 0.0;
            for (int m = 0; m <= j; ++m) s += ch[m * CP + r] * Li[m * K + j];
            dst[static_cast<int64_t>(j) * I + i0 + r] = s;
        }
    }
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cqr(const double* __restrict__ y, int I, int K,
                                                double* work, double* q64, T* q_out,
                                                uint32_t* flags) {
    extern __shared__ __align__(16) double shd[];
    double* G = shd;
    double* Li = G + K * K;
    double* ch = Li + K * K;
    __shared__ double diag0[RHOSVD_MAX_K];
    __shared__ double tau_s[RHOSVD_MAX_K], alpha_s[RHOSVD_MAX_K];
    __shared__ double red[kBlock / kWave];
    __shared__ int fail;
    __shared__ double shift_sh;

    // round 0 on Y, shifted if its Gram is not numerically positive definite
    cqr_gram(y, I, K, G, ch, 0.0);
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int j = 0; j < K; ++j) tr += G[j * K + j];
        shift_sh = 11.0 * (static_cast<double>(I) * K + static_cast<double>(K) * (K + 1)) *
                   1.1102230246251565e-16 * tr;
    }
    __syncthreads();
    bool ok = cqr_cholesky(G, K, diag0, &fail);
    bool shifted = false;
    if (!ok) {
        shifted = true;
        cqr_gram(y, I, K, G, ch, shift_sh);
        ok = cqr_cholesky(G, K, diag0, &fail);
    }
    if (ok) {
        const int rounds = shifted ? 3 : 2;
        // destination of round r: the last round writes q64
        double* dst0 = (rounds == 3) ? q64 : work;
        cqr_invert(G, K, Li);
        cqr_apply(y, I, K, Li, ch, dst0);
        double* cur = dst0;
        for (int r = 1; r < rounds && ok; ++r) {
            double* dst = (r == rounds - 1) ? q64 : (cur == q64 ? work : q64);
            cqr_gram(cur, I, K, G, ch, 0.0);
            ok = cqr_cholesky(G, K, diag0, &fail);
            if (!ok) break;
            cqr_invert(G, K, Li);
            cqr_apply(cur, I, K, Li, ch, dst);
            cur = dst;
        }
    }
    if (!ok) householder_qr(y, I, K, work, q64, tau_s, alpha_s, red);
    if (threadIdx.x == 0 && flags) {
        uint32_t f = shifted ? RHOSVD_FLAG_CQR_SHIFTED : 0u;
        if (!ok) f |= RHOSVD_FLAG_QR_HOUSEHOLDER;
        if (f) atomicOr(flags, f);
    }
    for (int e = threadIdx.x; e < I * K; e += kBlock) q_out[e] = static_cast<T>(q64[e]);
}

hipError_t launch_cqr_global(const double* y, int64_t I, int K, bool dbl, void* q_out,
                             double* q64, uint32_t* flags, hipStream_t s) {
    // work buffer lives right after q64 (the caller reserves 2 I K doubles)
    double* work = q64 + I * K;
    const size_t lds = (2 * static_cast<size_t>(K) * K + static_cast<size_t>(K) * (kCqrRows + 1)) *
                       sizeof(double);
    if (lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
    if (dbl)
        hipLaunchKernelGGL(k_cqr<double>, dim3(1), dim3(kBlock), lds, s, y, static_cast<int>(I), K,
                           work, q64, static_cast<double*>(q_out), flags);
    else
        hipLaunchKernelGGL(k_cqr<float>, dim3(1), dim3(kBlock), lds, s, y, static_cast<int>(I), K,
                           work, q64, static_cast<float*>(q_out), flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Omega test fill: out (J x K column-major) = Omega(seed, mode, tag).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_omega_fill(uint64_t seed, uint32_t mode, uint32_t tag, int64_t total,
                             T* __restrict__ out) {
    const int64_t nq = (total + 3) / 4;
    for (int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; q < nq;
         q += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        T z[4];
        normals4<T>(static_cast<uint64_t>(q), mode, tag, seed, z);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int64_t e = 4 * q + w;
            if (e < total) out[e] = z[w];
        }
    }
}

hipError_t launch_omega_fill(bool dbl, uint64_t seed, int mode, int tag, int64_t J, int K,
                             void* out, hipStream_t s) {
    const int64_t total = J * K;
    const int64_t nq = (total + 3) / 4;
    int64_t blocks = (nq + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    if (dbl)
        hipLaunchKernelGGL(k_omega_fill<double>, dim3(blocks), dim3(kBlock), 0, s, seed, mode, tag,
                           total, static_cast<double*>(out));
    else
        hipLaunchKernelGGL(k_omega_fill<float>, dim3(blocks), dim3(kBlock), 0, s, seed, mode, tag,
                           total, static_cast<float*>(out));
    return hipGetLastError();
}

// Several J x K Gaussian tables in one launch (the structured sketch's
// tables): table y = blockIdx.y holds the stream (seed, word, tag) as
// launch_omega_fill writes it.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_kr_fill(KrFill f) {
    const KrFill::Table& t = f.t[blockIdx.y];
    const int64_t total = t.J * static_cast<int64_t>(t.K);
    T* out = static_cast<T*>(t.out);
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; 4 * q < total;
         q += static_cast<int64_t>(gridDim.x) * kBlock) {
        T z[4];
        normals4<T>(static_cast<uint64_t>(q), t.word, f.tag, f.seed, z);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int64_t e = 4 * q + w;
            if (e < total) out[e] = z[w];
        }
    }
}

hipError_t launch_kr_fill(bool dbl, const KrFill& f, hipStream_t s) {
    if (f.count < 1 || f.count > KrFill::kMax) return hipErrorInvalidValue;
    int64_t most = 1;
    for (int i = 0; i < f.count; ++i) most = std::max<int64_t>(most, f.t[i].J * f.t[i].K);
    int64_t blocks = (most / 4 + kBlock) / kBlock;
    if (blocks > 256) blocks = 256;
    if (dbl)
        hipLaunchKernelGGL(k_kr_fill<double>, dim3(blocks, f.count), dim3(kBlock), 0, s, f);
    else
        hipLaunchKernelGGL(k_kr_fill<float>, dim3(blocks, f.count), dim3(kBlock), 0, s, f);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Report bookkeeping.
// ---------------------------------------------------------------------------
__global__ void k_report_init(rhosvd_report* rep, ReportInit ri, uint32_t init_flags) {
    const int tid = threadIdx.x;
    double* sg = &rep->sigma[0][0];
    for (int e = tid; e < RHOSVD_MAX_ORDER * RHOSVD_MAX_K; e += blockDim.x) sg[e] = 0.0;
    if (tid == 0) {
        rep->norm_x2 = 0.0;
        rep->norm_core2 = 0.0;
        rep->resid2 = 0.0;
        rep->order = ri.order;
        for (int n = 0; n < RHOSVD_MAX_ORDER; ++n) rep->k_used[n] = ri.k_used[n];
        rep->flags = init_flags;
    }
}

__global__ void k_report_mode(rhosvd_report* rep, int n, int k, int r) {
    for (int e = r + static_cast<int>(threadIdx.x); e < RHOSVD_MAX_K; e += blockDim.x) rep->sigma[n][e] = 0.0;
    if (threadIdx.x == 0) {
        rep->k_used[n] = k < 0 ? -k : k;
        if (k < 0) rep->flags |= RHOSVD_FLAG_K_CAPPED;
    }
}

hipError_t launch_report_mode(void* rep, int n, int k, int r, hipStream_t s) {
    hipLaunchKernelGGL(k_report_mode, dim3(1), dim3(kWave), 0, s, static_cast<rhosvd_report*>(rep),
                       n, k, r);
    return hipGetLastError();
}

hipError_t launch_report_init(void* rep, ReportInit ri, hipStream_t s) {
    uint32_t fl = 0;
    for (int n = 0; n < ri.order; ++n)
        if (ri.k_used[n] < 0) fl |= RHOSVD_FLAG_K_CAPPED;  // sign marks a capped K
    for (int n = 0; n < ri.order; ++n)
        if (ri.k_used[n] < 0) ri.k_used[n] = -ri.k_used[n];
    hipLaunchKernelGGL(k_report_init, dim3(1), dim3(kBlock), 0, s,
                       static_cast<rhosvd_report*>(rep), ri, fl);
    return hipGetLastError();
}

__global__ void k_copy_bytes(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
                             size_t n) {
    for (size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; e < n;
         e += static_cast<size_t>(gridDim.x) * blockDim.x)
        dst[e] = src[e];
}

hipError_t launch_copy_bytes(const void* src, void* dst, size_t n, hipStream_t s) {
    size_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy_bytes, dim3(blocks), dim3(kBlock), 0, s,
                       static_cast<const unsigned char*>(src), static_cast<unsigned char*>(dst), n);
    return hipGetLastError();
}

}  // namespace rh
