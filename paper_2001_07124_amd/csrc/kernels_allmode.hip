// Single-pass sketch of every mode (RP-HOSVD, Algorithm 6 step 3):
// Y_n = X_(n) Omega_n for n = 1..N from one read of X, without forming any
// unfolding (Section 5.1), plus the sum of squares of X.
//
// The tensor is cut into tiles of extents (b_1, ..., b_N) (about 4096
// elements).  A workgroup walks its tiles in a fixed order: the tile is
// staged in LDS once, then for every mode n its n-unfolding (b_n rows x
// prod_{m != n} b_m columns) is multiplied by the Omega_n rows of those
// columns, which the workgroup generates from the counter-based stream in
// chunks (Philox4x32-10 + Box-Muller, the row being the column's cyclic
// position).  Each (row i_n, column k) of a tile's product belongs to one
// thread, which adds it to the workgroup's copy of Y_n (all of Y_1..Y_N live
// in LDS); the copies are written once at the end and summed over
// workgroups in a fixed order, so the result is deterministic.  Each Omega_n
// row is generated once per tile that needs it: prod_{m != n} b_m K_n
// normals per tile, i.e. sum_n K_n / b_n per element of X.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"
#include "rhosvd.h"

namespace rh {

constexpr int kAmRows = 32;     // Omega rows per generated chunk

__device__ __forceinline__ int64_t am_decode(int64_t v, int64_t radix, int64_t* q) {
    *q = v / radix;
    return v - *q * radix;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_allmode(AllModeArgs a) {
    extern __shared__ __align__(16) unsigned char am_lds[];
    T* acc = reinterpret_cast<T*>(am_lds);                        // S
    T* tile = acc + a.S;                                          // TB
    T* om = tile + a.TB;                                          // kAmRows x KMAX
    int* colb = reinterpret_cast<int*>(om + kAmRows * a.KMAX);    // kAmRows column bases
    __shared__ double red[kBlock / kWave];
    const int tid = threadIdx.x;
    const int N = a.N;
    for (int64_t e = tid; e < a.S; e += kBlock) acc[e] = static_cast<T>(0);
    double ss = 0.0;
    for (int64_t tt = blockIdx.x; tt < a.ntiles; tt += gridDim.x) {
        // tile origin (first mode fastest over the tile grid)
        int64_t org[RHOSVD_MAX_ORDER];
        {
            int64_t v = tt;
            for (int m = 0; m < N; ++m) {
                int64_t q;
                org[m] = am_decode(v, a.ntile[m], &q) * a.b[m];
                v = q;
            }
        }
        __syncthreads();
        // stage the tile (zero outside the tensor), first local index fastest
        for (int64_t li = tid; li < a.TB; li += kBlock) {
            int64_t v = li, off = 0;
            bool in = true;
            for (int m = 0; m < N; ++m) {
                int64_t q;
                const int64_t lm = am_decode(v, a.b[m], &q);
                v = q;
                const int64_t g = org[m] + lm;
                in = in && g < a.dims[m];
                off += g * a.xs[m];
            }
            const T xv = in ? static_cast<const T*>(a.x)[off] : static_cast<T>(0);
            tile[li] = xv;
            ss += static_cast<double>(xv) * static_cast<double>(xv);
        }
        __syncthreads();
        for (int n = 0; n < N; ++n) {
            const int K = a.K[n];
            const int bn = a.b[n];
            const int64_t rows = a.TB / bn;             // tile columns of the n-unfolding
            const int64_t bsn = a.bs[n];
            const int nout = bn * K;
            T part[4] = {static_cast<T>(0), static_cast<T>(0), static_cast<T>(0), static_cast<T>(0)};
            for (int64_t r0 = 0; r0 < rows; r0 += kAmRows) {
                const int nr = rows - r0 < kAmRows ? static_cast<int>(rows - r0) : kAmRows;
                __syncthreads();
                // column bases and Omega rows of this chunk
                for (int e = tid; e < kAmRows * K; e += kBlock) {
                    const int r = e % kAmRows, k = e / kAmRows;
                    T w = static_cast<T>(0);
                    if (r < nr) {
                        // local coordinates of the other modes (natural order,
                        // first fastest); cyclic position of the global column
                        int64_t v = r0 + r, base = 0, l = 0, t = 0;
                        bool in = true;
                        for (int m = 0; m < N; ++m) {
                            if (m == n) continue;
                            int64_t q;
                            const int64_t lm = am_decode(v, a.b[m], &q);
                            v = q;
                            base += lm * a.bs[m];
                            const int64_t g = org[m] + lm;
                            in = in && g < a.dims[m];
                            if (m < n) l += g * a.xs[m];
                            else t += g * a.xs[m];
                        }
                        if (k == 0) colb[r] = static_cast<int>(base);
                        // t: the modes after n with their own strides, every
                        // term a multiple of the stride of mode n + 1
                        t = n + 1 < N ? t / a.xs[n + 1] : 0;
                        if (in) {
                            const uint64_t idx = static_cast<uint64_t>(k) * static_cast<uint64_t>(a.J[n]) +
                                                 static_cast<uint64_t>(t + a.T[n] * l);
                            T z[4];
                            normals4<T>(idx >> 2, static_cast<uint32_t>(n), a.tag, a.seed, z);
                            w = z[idx & 3];
                        }
                    } else if (k == 0) {
                        colb[r] = 0;
                    }
                    om[r * a.KMAX + k] = w;
                }
                __syncthreads();
                for (int j = 0; j < 4; ++j) {
                    const int o = tid + j * kBlock;
                    if (o < nout) {
                        const int il = o % bn, k = o / bn;
                        T s = part[j];
                        for (int r = 0; r < nr; ++r)
                            s = fma(tile[colb[r] + il * bsn], om[r * a.KMAX + k], s);
                        part[j] = s;
                    }
                }
            }
            // into the workgroup's Y_n (each entry has exactly one owner here)
            for (int j = 0; j < 4; ++j) {
                const int o = tid + j * kBlock;
                if (o < nout) {
                    const int il = o % bn, k = o / bn;
                    const int64_t gi = org[n] + il;
                    if (gi < a.dims[n]) acc[a.yoff[n] + gi + a.dims[n] * k] += part[j];
                }
            }
        }
    }
    __syncthreads();
    T* out = static_cast<T*>(a.part) + static_cast<int64_t>(blockIdx.x) * a.S;
    for (int64_t e = tid; e < a.S; e += kBlock) out[e] = acc[e];
    ss = wave_sum(ss);
    if ((tid & 63) == 0) red[tid >> 6] = ss;
    __syncthreads();
    if (tid == 0 && a.part_ss) {
        double t = 0.0;
        for (int q = 0; q < kBlock / kWave; ++q) t += red[q];
        a.part_ss[blockIdx.x] = t;
    }
}

// y[e] = sum_g part[g S + e] in order of g, e < S (all modes at once).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_allmode_reduce(const T* __restrict__ part, int G,
                                                           int64_t S, double* __restrict__ y) {
    const int64_t e = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x;
    if (e >= S) return;
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += static_cast<double>(part[static_cast<int64_t>(g) * S + e]);
    y[e] = s;
}

bool plan_allmode(int N, const int64_t* dims, const int* K, int num_cu, int elem, AllModeArgs* a) {
    if (N < 2 || N > RHOSVD_MAX_ORDER) return false;
    *a = AllModeArgs{};
    a->N = N;
    int kmax = 1;
    for (int n = 0; n < N; ++n) {
        if (K[n] < 1 || K[n] > 64 || dims[n] < 1) return false;
        if (K[n] > kmax) kmax = K[n];
    }
    a->KMAX = kmax;
    // tile extents: the largest B <= 16 with B^N <= 4096, capped by each
    // extent (a thread then owns at most 16 K / 256 <= 4 outputs per mode)
    int B = 1;
    while (B < 16) {
        int64_t p = 1;
        for (int n = 0; n < N; ++n) p *= B + 1;
        if (p > 4096) break;
        ++B;
    }
    int64_t TB = 1, nt = 1, S = 0, xs = 1;
    for (int n = 0; n < N; ++n) {
        a->dims[n] = dims[n];
        a->K[n] = K[n];
        a->b[n] = static_cast<int>(dims[n] < B ? dims[n] : B);
        a->bs[n] = TB;
        TB *= a->b[n];
        a->ntile[n] = (dims[n] + a->b[n] - 1) / a->b[n];
        nt *= a->ntile[n];
        a->xs[n] = xs;
        xs *= dims[n];
        a->yoff[n] = S;
        S += dims[n] * K[n];
    }
    // per mode: J_n and T_n of the cyclic column position c = t + T_n l
    // (t over the modes after n, l over those before)
    for (int n = 0; n < N; ++n) {
        int64_t st = 1, sl = 1;
        for (int m = n + 1; m < N; ++m) st *= dims[m];
        for (int m = 0; m < n; ++m) sl *= dims[m];
        a->T[n] = st;
        a->J[n] = st * sl;
    }
    a->TB = TB;
    a->S = S;
    a->ntiles = nt;
    int64_t g = static_cast<int64_t>(num_cu) * 2;
    if (g > nt) g = nt;
    a->grid = static_cast<int>(g < 1 ? 1 : g);
    a->lds_bytes = static_cast<size_t>(S + TB + static_cast<int64_t>(kAmRows) * kmax) * elem +
                   kAmRows * sizeof(int);
    return a->lds_bytes + kStaticLdsMargin <= kLdsLimit;
}

hipError_t launch_allmode(bool dbl, const AllModeArgs& a, hipStream_t s) {
    if (dbl)
        hipLaunchKernelGGL(k_allmode<double>, dim3(a.grid), dim3(kBlock), a.lds_bytes, s, a);
    else
        hipLaunchKernelGGL(k_allmode<float>, dim3(a.grid), dim3(kBlock), a.lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_allmode_reduce(bool dbl, const AllModeArgs& a, double* y, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((a.S + kBlock - 1) / kBlock));
    if (dbl)
        hipLaunchKernelGGL(k_allmode_reduce<double>, grid, dim3(kBlock), 0, s,
                           static_cast<const double*>(a.part), a.grid, a.S, y);
    else
        hipLaunchKernelGGL(k_allmode_reduce<float>, grid, dim3(kBlock), 0, s,
                           static_cast<const float*>(a.part), a.grid, a.S, y);
    return hipGetLastError();
}

}  // namespace rh
