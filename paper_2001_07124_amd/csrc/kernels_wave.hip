// Wave-private streaming kernels for FP32 tensors (gfx950).
//
// Each wave owns whole blocks of 16 consecutive unfolding columns of the
// current tensor S_(n) (an (L, I, T) view, see kernels.hpp) and keeps the
// block in registers in the layout the matrix cores read for S^T Q: lane
// (c = l % 16, g = l / 16) holds S(16 f + 4 g + e, c), e = 0..3, for every
// 16-row block f.  For L = 1 that is one 16-byte load per row block.
//
//   P2  Z = S_blk^T M        (16 x K)  A = the block, B = M fragments (LDS)
//   P1  Y += S_blk W         (I x K)   A = the block transposed through a
//                                      wave-private LDS scratch, B = W
// The accumulator layout of P2 (lane (r, g) holds Z(4 g + e, r)) is exactly
// the B-operand layout of P1 and the A/B layout of the Gram Z^T Z, so the
// power step and the Gram need no data movement between the two products.
// Workgroups are 4 independent waves; the only barriers are at the start
// (M fragments) and at the end (cross-wave reduction of the partials).
//
// Tall modes (RS = 4, 256 < I <= 64 IBT): the four waves of a workgroup
// share each block, wave w holding the row blocks w IBW .. (w + 1) IBW - 1.
// The sketch needs no exchange (each wave accumulates its own rows of Y);
// in the power step and the mode-n product the waves' partial Z = S_w^T M_w
// are summed through LDS in wave order, one barrier per block (two exchange
// buffers alternate, so a wave never overwrites a buffer another still
// reads), and every wave continues with the same Z.  Wave 0 writes the
// mode-n product and forms its Gram.
//
// Matrix-core precision (CompType):
//   CT_F32     four v_mfma_f32_16x16x4_f32 per 16x16x16 step
//   CT_BF16    one v_mfma_f32_16x16x16_bf16 (inputs rounded to bf16)
//   CT_BF16X3  split x = hi + lo (both bf16), hi*hi + hi*lo + lo*hi
//   CT_BF16X2  bf16 tensor against a split operand: hi*hi + hi*lo.  Rounding
//              the small operand (Q, U) would change the captured energy
//              ||M^T S||^2 at first order (the large singular values multiply
//              the rounding error); rounding the streamed tensor does not.
// Accumulation is always FP32.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"
#include "rhosvd.h"

namespace rh {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

template <int CT>
struct FragT;
template <>
struct FragT<CT_F32> {
    f32x4 v;
};
template <>
struct FragT<CT_BF16> {
    bf16x4 hi;
};
template <>
struct FragT<CT_BF16X3> {
    bf16x4 hi, lo;
};

template <int CT>
__device__ __forceinline__ FragT<CT> make_frag(f32x4 x);
template <>
__device__ __forceinline__ FragT<CT_F32> make_frag<CT_F32>(f32x4 x) {
    FragT<CT_F32> f;
    f.v = x;
    return f;
}
template <>
__device__ __forceinline__ FragT<CT_BF16> make_frag<CT_BF16>(f32x4 x) {
    FragT<CT_BF16> f;
#pragma unroll
    for (int e = 0; e < 4; ++e) f.hi[e] = static_cast<__bf16>(x[e]);
    return f;
}
template <>
__device__ __forceinline__ FragT<CT_BF16X3> make_frag<CT_BF16X3>(f32x4 x) {
    FragT<CT_BF16X3> f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const __bf16 h = static_cast<__bf16>(x[e]);
        f.hi[e] = h;
        f.lo[e] = static_cast<__bf16>(x[e] - static_cast<float>(h));
    }
    return f;
}

__device__ __forceinline__ f32x4 mma(const FragT<CT_F32>& a, const FragT<CT_F32>& b, f32x4 c) {
#pragma unroll
    for (int e = 0; e < 4; ++e) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[e], b.v[e], c, 0, 0, 0);
    return c;
}
__device__ __forceinline__ f32x4 mma(const FragT<CT_BF16>& a, const FragT<CT_BF16>& b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.hi, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma(const FragT<CT_BF16X3>& a, const FragT<CT_BF16X3>& b,
                                     f32x4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.lo, b.hi, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.lo, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.hi, c, 0, 0, 0);
}
// bf16 data against a split (hi + lo) operand: the streamed tensor is
// rounded once, the small factor-like operand keeps ~16 mantissa bits.
__device__ __forceinline__ f32x4 mma(const FragT<CT_BF16>& a, const FragT<CT_BF16X3>& b, f32x4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.lo, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.hi, c, 0, 0, 0);
}

// Compute type -> fragment types of the streamed data (A side) and of the
// K-wide operand (B side: M, Z or Omega).
template <int CT>
struct Sides {
    static constexpr int data = CT;
    static constexpr int op = CT;
};
template <>
struct Sides<CT_BF16X2> {
    static constexpr int data = CT_BF16;
    static constexpr int op = CT_BF16X3;
};

// Transpose of one 16x16 block through the wave's LDS scratch (row pitch
// 16 elements): write the P2 layout, read the P1 layout (lane (i, g) gets
// S(i, 4 g + e)).
__device__ __forceinline__ void scr_put(float* s, int f, int quad, int l16, const FragT<CT_F32>& x) {
#pragma unroll
    for (int e = 0; e < 4; ++e) s[(16 * f + 4 * quad + e) * 16 + l16] = x.v[e];
}
__device__ __forceinline__ FragT<CT_F32> scr_get(const float* s, int f, int quad, int l16) {
    FragT<CT_F32> x;
    x.v = *reinterpret_cast<const f32x4*>(s + (16 * f + l16) * 16 + 4 * quad);
    return x;
}
__device__ __forceinline__ void scr_put(__bf16* s, int f, int quad, int l16, const FragT<CT_BF16>& x) {
#pragma unroll
    for (int e = 0; e < 4; ++e) s[(16 * f + 4 * quad + e) * 16 + l16] = x.hi[e];
}
__device__ __forceinline__ FragT<CT_BF16> scr_get(const __bf16* s, int f, int quad, int l16) {
    FragT<CT_BF16> x;
    x.hi = *reinterpret_cast<const bf16x4*>(s + (16 * f + l16) * 16 + 4 * quad);
    return x;
}

template <int CT>
struct ScrT {
    typedef __bf16 elem;
    static constexpr int planes = (CT == CT_BF16X3) ? 2 : 1;
};
template <>
struct ScrT<CT_F32> {
    typedef float elem;
    static constexpr int planes = 1;
};

template <int CT>
__device__ __forceinline__ void scr_put_frag(unsigned char* base, int plane_elems, int f, int quad,
                                             int l16, const FragT<CT>& x);
template <>
__device__ __forceinline__ void scr_put_frag<CT_F32>(unsigned char* base, int, int f, int quad,
                                                     int l16, const FragT<CT_F32>& x) {
    scr_put(reinterpret_cast<float*>(base), f, quad, l16, x);
}
template <>
__device__ __forceinline__ void scr_put_frag<CT_BF16>(unsigned char* base, int, int f, int quad,
                                                      int l16, const FragT<CT_BF16>& x) {
    scr_put(reinterpret_cast<__bf16*>(base), f, quad, l16, x);
}
template <>
__device__ __forceinline__ void scr_put_frag<CT_BF16X3>(unsigned char* base, int plane_elems, int f,
                                                        int quad, int l16,
                                                        const FragT<CT_BF16X3>& x) {
    __bf16* s = reinterpret_cast<__bf16*>(base);
    FragT<CT_BF16> h, l;
    h.hi = x.hi;
    l.hi = x.lo;
    scr_put(s, f, quad, l16, h);
    scr_put(s + plane_elems, f, quad, l16, l);
}

template <int CT>
__device__ __forceinline__ FragT<CT> scr_get_frag(const unsigned char* base, int plane_elems, int f,
                                                  int quad, int l16);
template <>
__device__ __forceinline__ FragT<CT_F32> scr_get_frag<CT_F32>(const unsigned char* base, int, int f,
                                                              int quad, int l16) {
    return scr_get(reinterpret_cast<const float*>(base), f, quad, l16);
}
template <>
__device__ __forceinline__ FragT<CT_BF16> scr_get_frag<CT_BF16>(const unsigned char* base, int,
                                                                int f, int quad, int l16) {
    return scr_get(reinterpret_cast<const __bf16*>(base), f, quad, l16);
}
template <>
__device__ __forceinline__ FragT<CT_BF16X3> scr_get_frag<CT_BF16X3>(const unsigned char* base,
                                                                    int plane_elems, int f,
                                                                    int quad, int l16) {
    const __bf16* s = reinterpret_cast<const __bf16*>(base);
    FragT<CT_BF16X3> x;
    x.hi = scr_get(s, f, quad, l16).hi;
    x.lo = scr_get(s + plane_elems, f, quad, l16).hi;
    return x;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_wave_barrier();
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

// Omega(j, k) for the four consecutive columns j = jb .. jb+3 at row k of the
// (J x K) test matrix: linear indices e = k J + j (see normals4).
__device__ __forceinline__ f32x4 omega4(uint64_t e0, uint32_t mode, uint32_t tag, uint64_t seed,
                                        bool aligned) {
    float z[4];
    normals4<float>(e0 >> 2, mode, tag, seed, z);
    f32x4 w;
    if (aligned) {
        w[0] = z[0]; w[1] = z[1]; w[2] = z[2]; w[3] = z[3];
    } else {
        float z2[4];
        normals4<float>((e0 >> 2) + 1, mode, tag, seed, z2);
        const int off = static_cast<int>(e0 & 3);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = off + e;
            w[e] = k < 4 ? z[k] : z2[k - 4];
        }
    }
    return w;
}

// One block of 16 unfolding columns in the P2 layout: lane (c, g) gets
// S(16 f + 4 g + e, j0 + c), zero outside the tensor.
template <int MAXIB>
__device__ __forceinline__ void load_block(const WGeom& g, const float* __restrict__ src,
                                           int64_t blk, int l16, int quad, f32x4 (&sf)[MAXIB],
                                           int fb0, int IB) {
    const int I = static_cast<int>(g.I);
    const int64_t L = g.L, J = g.J;
    const int64_t j0 = blk * 16;
    const bool cok = j0 + l16 < J;
    if (g.vec4) {
        // buffer loads over the block's 16 contiguous columns: one uniform
        // 64-bit base, 32-bit lane offsets, columns past J read as zero
        // (outside the range); 16 I floats < 2^31 bytes for I <= 512
        const int64_t ncol = J - j0 < 16 ? (J > j0 ? J - j0 : 0) : 16;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(src + j0 * static_cast<int64_t>(I)), static_cast<short>(0),
            static_cast<int>(ncol * I * 4), 0x00020000);
        const int cbase = l16 * I * 4;
#pragma unroll
        for (int f = 0; f < MAXIB; ++f) {
            if (f < IB) {
                const int i0 = 16 * (fb0 + f) + 4 * quad;
                const f32x4 v = __builtin_bit_cast(
                    f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, cbase + 4 * i0, 0, 0));
                sf[f] = i0 < I ? v : zero4<f32x4>();
            }
        }
    } else {
        int64_t colbase = 0;
        if (cok) {
            const int64_t j = j0 + l16;
            const int64_t t = j / L;
            colbase = (j - t * L) + L * static_cast<int64_t>(I) * t;
        }
#pragma unroll
        for (int f = 0; f < MAXIB; ++f) {
            if (f < IB) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int i = 16 * (fb0 + f) + 4 * quad + e;
                    sf[f][e] = (cok && i < I) ? src[colbase + L * i] : 0.0f;
                }
            }
        }
    }
}

// IBT / NBT bound the row blocks of the block and the 16-column blocks of
// the K-wide operand; EXACT variants fix IB = IBT and NB = NBT at compile
// time (no masks, no spare accumulators).
template <int OP, int CT, int IBT, int NBT, bool EXACT, int RS>
__device__ __forceinline__ void wave_body(const WGeom& g, const StreamArgs& a, int want_ss,
                                          int want_gram, int bidx, int nwg) {
    constexpr int DCT = Sides<CT>::data;    // streamed tensor
    constexpr int OCT = Sides<CT>::op;      // K-wide operand
    typedef FragT<DCT> F;
    typedef FragT<OCT> FO;
    constexpr int GCT = (CT == CT_F32) ? CT_F32 : CT_BF16X3;   // Gram precision
    typedef FragT<GCT> FG;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, quad = lane >> 4;
    // IB: row blocks of the mode; this wave holds nf of them from fb0 on
    const int IB = EXACT ? IBT * RS : g.IB;
    const int NB = EXACT ? NBT : g.NB;
    const int IBW = RS == 1 ? IB : (EXACT ? IBT : g.IBW);
    const int fb0 = RS == 1 ? 0 : wave * IBW;
    const int nf = RS == 1 ? IB : (IB - fb0 < IBW ? (IB - fb0 > 0 ? IB - fb0 : 0) : IBW);
    const int K = g.K, I = static_cast<int>(g.I);
    const int64_t L = g.L, J = g.J;

    FO* qfr = reinterpret_cast<FO*>(smem);
    unsigned char* scr = smem + g.q_bytes + static_cast<size_t>(wave) * g.scr_bytes;
    const int plane_elems = IBW * 256;

    // M fragments (B operand of P2): fragment (f, nb), lane (r, g) holds
    // M(16 f + 4 g + e, 16 nb + r).
    if (OP != OP_SKETCH) {
        const float* __restrict__ m = static_cast<const float*>(a.mat);
        for (int idx = tid; idx < IB * NB * 64; idx += kBlock) {
            const int ln = idx & 63, fn = idx >> 6;
            const int f = fn / NB, nb = fn - f * NB;
            const int r = 16 * nb + (ln & 15), gq = ln >> 4;
            f32x4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 16 * f + 4 * gq + e;
                float x = 0.0f;
                if (i < I && r < K) x = m ? m[static_cast<int64_t>(r) * I + i] : (i == r ? 1.0f : 0.0f);
                v[e] = x;
            }
            qfr[idx] = make_frag<OCT>(v);
        }
        __syncthreads();
    }

    constexpr int AI = (OP == OP_TTM) ? 1 : IBT;    // Y accumulators (sketch, power)
    constexpr int AN = (OP == OP_TTM) ? 1 : NBT;
    constexpr int GN = (OP == OP_TTM) ? NBT : 1;    // Gram accumulators (TTM)
    f32x4 acc[AI][AN];
    f32x4 accg[GN][GN];
#pragma unroll
    for (int f = 0; f < AI; ++f)
#pragma unroll
        for (int nb = 0; nb < AN; ++nb) acc[f][nb] = zero4<f32x4>();
#pragma unroll
    for (int f = 0; f < GN; ++f)
#pragma unroll
        for (int nb = 0; nb < GN; ++nb) accg[f][nb] = zero4<f32x4>();
    double ss = 0.0;

    const float* __restrict__ src = static_cast<const float*>(a.src);
    // RS = 1: one block per wave; RS = 4: one block per workgroup
    const int64_t wid = RS == 1 ? static_cast<int64_t>(bidx) * (kBlock / kWave) + wave
                                : static_cast<int64_t>(bidx);
    const int64_t nw = RS == 1 ? static_cast<int64_t>(nwg) * (kBlock / kWave)
                               : static_cast<int64_t>(nwg);
    const bool jal = (J & 3) == 0;
    f32x4* xr = reinterpret_cast<f32x4*>(smem + g.xr_off);   // [2][RS][NBT][64] when RS > 1
    int par = 0;

    // software pipeline: the next block's loads are in flight while this
    // block is processed (one wave per SIMD, so the wave hides its own latency)
    f32x4 sf[IBT], sfn[IBT];
    if (wid < g.nblocks) load_block<IBT>(g, src, wid, l16, quad, sf, fb0, nf);
    for (int64_t blk = wid; blk < g.nblocks; blk += nw) {
        const int64_t j0 = blk * 16;
        const int cv = static_cast<int>(J - j0 < 16 ? J - j0 : 16);
        const bool cok = l16 < cv;
        if (blk + nw < g.nblocks) load_block<IBT>(g, src, blk + nw, l16, quad, sfn, fb0, nf);

        if (want_ss) {
            float part = 0.0f;
#pragma unroll
            for (int f = 0; f < IBT; ++f)
                if (f < nf)
#pragma unroll
                    for (int e = 0; e < 4; ++e) part = fmaf(sf[f][e], sf[f][e], part);
            ss += static_cast<double>(part);
        }

        // ---- per row block: P2 products Z += S_f^T M_f and the transpose scratch
        f32x4 z[NBT];
#pragma unroll
        for (int nb = 0; nb < NBT; ++nb) z[nb] = zero4<f32x4>();
#pragma unroll
        for (int f = 0; f < IBT; ++f) {
            if (f < nf) {
                const F sbf = make_frag<DCT>(sf[f]);
                if (OP != OP_SKETCH) {
#pragma unroll
                    for (int nb = 0; nb < NBT; ++nb)
                        if (nb < NB) z[nb] = mma(sbf, qfr[((fb0 + f) * NB + nb) * 64 + lane], z[nb]);
                }
                if (OP != OP_TTM) scr_put_frag<DCT>(scr, plane_elems, f, quad, l16, sbf);
            }
        }
        if constexpr (RS > 1 && OP != OP_SKETCH) {
            // Z = sum over the waves' rows, in wave order
            f32x4* xb = xr + static_cast<size_t>(par) * RS * NBT * 64;
#pragma unroll
            for (int nb = 0; nb < NBT; ++nb)
                if (nb < NB) xb[(wave * NBT + nb) * 64 + lane] = z[nb];
            __syncthreads();
#pragma unroll
            for (int nb = 0; nb < NBT; ++nb) {
                if (nb < NB) {
                    f32x4 t = xb[nb * 64 + lane];
#pragma unroll
                    for (int w = 1; w < RS; ++w) {
                        const f32x4 o = xb[(w * NBT + nb) * 64 + lane];
#pragma unroll
                        for (int e = 0; e < 4; ++e) t[e] += o[e];
                    }
                    z[nb] = t;
                }
            }
            par ^= 1;
        }

        // ---- P1: Y += S_blk W with W = Omega (sketch) or Z (power step)
        if (OP != OP_TTM) {
            FO wb[NBT];
#pragma unroll
            for (int nb = 0; nb < NBT; ++nb) {
                if (nb < NB) {
                    if (OP == OP_SKETCH) {
                        const int r = 16 * nb + l16;
                        f32x4 w = zero4<f32x4>();
                        if (r < K && L > 1) {
                            // generator rows are not consecutive along the block
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int64_t j = j0 + 4 * quad + e;
                                w[e] = j >= J ? 0.0f
                                       : a.kr.nq ? kr_entry<float>(a.kr, j, r)
                                                 : omega_entry<float>(a.seed, a.mode, a.tag, j, r, L, g.T, J);
                            }
                        } else if (r < K) {
                            const uint64_t e0 = static_cast<uint64_t>(r) * static_cast<uint64_t>(J) +
                                                static_cast<uint64_t>(j0 + 4 * quad);
                            if (a.kr.nq) {
                                float t4[4];
                                kr_entry4<float>(a.kr, j0 + 4 * quad, r, t4);
#pragma unroll
                                for (int e = 0; e < 4; ++e) w[e] = t4[e];
                            } else {
                                w = omega4(e0, a.mode, a.tag, a.seed, jal);
                            }
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (4 * quad + e >= cv) w[e] = 0.0f;
                        }
                        wb[nb] = make_frag<OCT>(w);
                    } else {
                        wb[nb] = make_frag<OCT>(z[nb]);
                    }
                }
            }
            wave_lds_sync();
#pragma unroll
            for (int f = 0; f < IBT; ++f) {
                if (f < nf) {
                    const F t = scr_get_frag<DCT>(scr, plane_elems, f, quad, l16);
#pragma unroll
                    for (int nb = 0; nb < NBT; ++nb)
                        if (nb < NB) acc[f][nb] = mma(t, wb[nb], acc[f][nb]);
                }
            }
            wave_lds_sync();
        }

        // ---- mode-n product output (folded) and its Gram
        if (OP == OP_TTM && (RS == 1 || wave == 0)) {
            if (want_gram) {
                FG zg[NBT];
#pragma unroll
                for (int nb = 0; nb < NBT; ++nb)
                    if (nb < NB) zg[nb] = make_frag<GCT>(z[nb]);
#pragma unroll
                for (int nb = 0; nb < NBT; ++nb)
#pragma unroll
                    for (int nb2 = 0; nb2 < NBT; ++nb2)
                        if (nb < NB && nb2 < NB) accg[nb][nb2] = mma(zg[nb], zg[nb2], accg[nb][nb2]);
            }
            float* __restrict__ out = static_cast<float*>(a.out);
            if (L == 1 && a.out_t) {
#pragma unroll
                for (int nb = 0; nb < NBT; ++nb) {
                    const int r = 16 * nb + l16;
                    if (nb < NB && r < K) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int cc = 4 * quad + e;
                            if (cc < cv) out[static_cast<int64_t>(r) * J + j0 + cc] = z[nb][e];
                        }
                    }
                }
            } else if (L == 1) {
#pragma unroll
                for (int nb = 0; nb < NBT; ++nb) {
                    const int r = 16 * nb + l16;
                    if (nb < NB && r < K) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int cc = 4 * quad + e;
                            if (cc < cv) out[(j0 + cc) * static_cast<int64_t>(K) + r] = z[nb][e];
                        }
                    }
                }
            } else {
                // stage Z through the scratch so that lanes write runs along l
                float* st = reinterpret_cast<float*>(scr);
#pragma unroll
                for (int nb = 0; nb < NBT; ++nb)
                    if (nb < NB)
#pragma unroll
                        for (int e = 0; e < 4; ++e) st[(16 * nb + l16) * 17 + 4 * quad + e] = z[nb][e];
                wave_lds_sync();
                if (cok) {
                    const int64_t j = j0 + l16;
                    const int64_t t = j / L;
                    float* __restrict__ op = out + (j - t * L) + L * static_cast<int64_t>(K) * t;
                    for (int r = quad; r < K; r += 4) op[L * r] = st[r * 17 + l16];
                }
                wave_lds_sync();
            }
        }
#pragma unroll
        for (int f = 0; f < IBT; ++f) sf[f] = sfn[f];
    }

    // ---- cross-wave reduction (fixed order) and the per-workgroup partials
    __syncthreads();
    float* red = reinterpret_cast<float*>(smem);
    const size_t gidx = static_cast<size_t>(bidx);
    const int I_pad = IB * 16, K_pad = NB * 16;
    if (OP != OP_TTM && RS > 1) {
        // the waves hold disjoint rows: each writes its own
#pragma unroll
        for (int f = 0; f < AI; ++f)
#pragma unroll
            for (int nb = 0; nb < AN; ++nb)
                if (f < nf && nb < NB)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        red[(16 * nb + l16) * I_pad + 16 * (fb0 + f) + 4 * quad + e] = acc[f][nb][e];
        __syncthreads();
        float* __restrict__ py = static_cast<float*>(a.part_y) + gidx * K_pad * I_pad;
        for (int e = tid; e < K_pad * I_pad; e += kBlock) py[e] = red[e];
    } else if (OP != OP_TTM) {
        for (int w = 0; w < kBlock / kWave; ++w) {
            if (wave == w) {
#pragma unroll
                for (int f = 0; f < AI; ++f)
#pragma unroll
                    for (int nb = 0; nb < AN; ++nb)
                        if (f < IB && nb < NB)
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int idx = (16 * nb + l16) * I_pad + 16 * f + 4 * quad + e;
                                red[idx] = (w == 0 ? 0.0f : red[idx]) + acc[f][nb][e];
                            }
            }
            __syncthreads();
        }
        float* __restrict__ py = static_cast<float*>(a.part_y) + gidx * K_pad * I_pad;
        for (int e = tid; e < K_pad * I_pad; e += kBlock) py[e] = red[e];
    }
    if (OP == OP_TTM && want_gram) {
        for (int w = 0; w < kBlock / kWave; ++w) {
            if (wave == w) {
#pragma unroll
                for (int nb = 0; nb < GN; ++nb)
#pragma unroll
                    for (int nb2 = 0; nb2 < GN; ++nb2)
                        if (nb < NB && nb2 < NB)
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int idx = (16 * nb2 + l16) * K_pad + 16 * nb + 4 * quad + e;
                                red[idx] = (w == 0 ? 0.0f : red[idx]) + accg[nb][nb2][e];
                            }
            }
            __syncthreads();
        }
        float* __restrict__ pg = static_cast<float*>(a.part_g) + gidx * K_pad * K_pad;
        for (int e = tid; e < K_pad * K_pad; e += kBlock) pg[e] = red[e];
    }
    if (want_ss) {
        __shared__ double rs[kBlock / kWave];
        ss = wave_sum(ss);
        if (lane == 0) rs[wave] = ss;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w) s += rs[w];
            a.part_ss[gidx] = s;
        }
    }
}

template <int OP, int CT, int IBT, int NBT, bool EXACT, int RS>
__global__ __launch_bounds__(kBlock, 1) void k_wave(WGeom g, StreamArgs a, int want_ss,
                                                    int want_gram) {
    wave_body<OP, CT, IBT, NBT, EXACT, RS>(g, a, want_ss, want_gram, blockIdx.x, gridDim.x);
}

// Many problems: job blockIdx.y on workgroups 0 .. units - 1 of grid x.
template <int OP, int CT, int IBT, int NBT>
__global__ __launch_bounds__(kBlock, 1) void k_wave_batch(const WaveJob* __restrict__ jobs) {
    const WaveJob& j = jobs[blockIdx.y];      // read in place: uniform, scalar loads
    if (static_cast<int>(blockIdx.x) >= j.units) return;
    wave_body<OP, CT, IBT, NBT, false, 1>(j.g, j.a, j.want_ss, j.want_gram, blockIdx.x, j.units);
}

// ---------------------------------------------------------------------------
// Planning and dispatch.
// ---------------------------------------------------------------------------
// Shapes with exact instantiations (row blocks, operand column blocks), then
// bounded generic ones.  C3-like modes use (13, 3) (I = 200, K = 35) and the
// truncation (3, 2) (I = K = 35, R = 25).
static const int kExact[][2] = {{13, 3}, {3, 2}, {13, 2}, {7, 1}};
static const int kGeneric[][2] = {{4, 4}, {8, 4}, {16, 2}, {16, 3}, {16, 4}};
constexpr int kNumExact = 4, kNumGeneric = 5;
// Tall modes, four waves per block (row blocks per wave, operand blocks):
// an exact 500-row case (IB = 32, NB = 2), then bounded generic ones.
static const int kTall[][3] = {{8, 2, 1}, {8, 2, 0}, {6, 3, 0}};
constexpr int kNumTall = 3;
constexpr int kTallRS = 4;
constexpr int kTallVariant0 = 9;    // variant index of kTall[0]

static bool plan_wave_tall(int op, int ct, int64_t L, int64_t I, int64_t T, int K, int num_cu,
                           WGeom* g);

bool plan_wave(int op, int ct, int64_t L, int64_t I, int64_t T, int K, int num_cu, WGeom* g) {
    if (L < 1 || I < 1 || T < 1 || K < 1) return false;
    const int IB = static_cast<int>((I + 15) / 16), NB = (K + 15) / 16;
    int var = -1;
    for (int v = 0; v < kNumExact; ++v)
        if (IB == kExact[v][0] && NB == kExact[v][1]) var = v;
    if (var < 0)
        for (int v = 0; v < kNumGeneric; ++v)
            if (IB <= kGeneric[v][0] && NB <= kGeneric[v][1]) {
                var = kNumExact + v;
                break;
            }
    if (var < 0) return plan_wave_tall(op, ct, L, I, T, K, num_cu, g);
    g->rs = 1;
    g->IBW = IB;
    g->xr_off = 0;
    g->L = L;
    g->I = I;
    g->T = T;
    g->J = L * T;
    g->K = K;
    g->IB = IB;
    g->NB = NB;
    g->ct = ct;
    g->variant = var;
    const size_t frag = (ct == CT_BF16) ? 8 : 16;               // operand fragment per lane
    g->q_bytes = (op != OP_SKETCH) ? static_cast<size_t>(IB) * NB * 64 * frag : 0;
    const size_t comp = (ct == CT_F32) ? 4 : 2;
    const size_t planes = (ct == CT_BF16X3) ? 2 : 1;
    size_t scr = 0;
    if (op != OP_TTM) scr = static_cast<size_t>(IB) * 256 * comp * planes;   // transpose
    else if (L > 1) scr = static_cast<size_t>(NB) * 16 * 17 * 4;             // output staging
    g->scr_bytes = (scr + 15) / 16 * 16;
    size_t lds = g->q_bytes + 4 * g->scr_bytes;
    size_t red = static_cast<size_t>(IB) * 16 * NB * 16 * 4;
    const size_t redg = static_cast<size_t>(NB) * 16 * NB * 16 * 4;
    if (redg > red) red = redg;
    if (red > lds) lds = red;
    if (lds + kStaticLdsMargin > kLdsLimit) return false;
    g->lds_bytes = lds;
    g->nblocks = (g->J + 15) / 16;
    const int64_t wgs = (g->nblocks + 3) / 4;
    const int64_t cap = num_cu > 0 ? num_cu : 256;
    g->grid = static_cast<int>(wgs < cap ? wgs : cap);
    g->vec4 = (L == 1 && I % 4 == 0) ? 1 : 0;
    return true;
}

static bool plan_wave_tall(int op, int ct, int64_t L, int64_t I, int64_t T, int K, int num_cu,
                           WGeom* g) {
    const int IB = static_cast<int>((I + 15) / 16), NB = (K + 15) / 16;
    const int ibw = (IB + kTallRS - 1) / kTallRS;
    const size_t frag = (ct == CT_BF16) ? 8 : 16;
    const size_t comp = (ct == CT_F32) ? 4 : 2;
    const size_t planes = (ct == CT_BF16X3) ? 2 : 1;
    for (int v = 0; v < kNumTall; ++v) {
        const int ibt = kTall[v][0], nbt = kTall[v][1];
        const bool exact = kTall[v][2] != 0;
        if (exact ? (IB != kTallRS * ibt || NB != nbt) : (ibw > ibt || NB > nbt)) continue;
        const size_t q_bytes = (op != OP_SKETCH) ? static_cast<size_t>(IB) * NB * 64 * frag : 0;
        size_t scr = 0;
        if (op != OP_TTM) scr = static_cast<size_t>(ibw) * 256 * comp * planes;
        else if (L > 1) scr = static_cast<size_t>(NB) * 16 * 17 * 4;
        const size_t scr_bytes = (scr + 15) / 16 * 16;
        const size_t xr_off = q_bytes + 4 * scr_bytes;
        const size_t xr = (op != OP_SKETCH) ? static_cast<size_t>(2) * kTallRS * nbt * 64 * 16 : 0;
        size_t lds = xr_off + xr;
        size_t red = static_cast<size_t>(IB) * 16 * NB * 16 * 4;
        const size_t redg = static_cast<size_t>(NB) * 16 * NB * 16 * 4;
        if (redg > red) red = redg;
        if (red > lds) lds = red;
        if (lds + kStaticLdsMargin > kLdsLimit) continue;
        g->L = L;
        g->I = I;
        g->T = T;
        g->J = L * T;
        g->K = K;
        g->IB = IB;
        g->NB = NB;
        g->ct = ct;
        g->variant = kTallVariant0 + v;
        g->q_bytes = q_bytes;
        g->scr_bytes = scr_bytes;
        g->lds_bytes = lds;
        g->rs = kTallRS;
        g->IBW = exact ? ibt : ibw;
        g->xr_off = xr_off;
        g->nblocks = (g->J + 15) / 16;
        const int64_t cap = num_cu > 0 ? num_cu : 256;
        g->grid = static_cast<int>(g->nblocks < cap ? g->nblocks : cap);
        g->vec4 = (L == 1 && I % 4 == 0) ? 1 : 0;
        return true;
    }
    return false;
}

template <int OP, int CT, int MI, int MN, bool EX, int RS = 1>
static hipError_t launch_wave_t(const WGeom& g, const StreamArgs& a, hipStream_t s) {
    const int want_ss = a.part_ss != nullptr;
    const int want_gram = a.part_g != nullptr;
    auto fn = k_wave<OP, CT, MI, MN, EX, RS>;
    hipLaunchKernelGGL(fn, dim3(g.grid), dim3(kBlock), g.lds_bytes, s, g, a, want_ss, want_gram);
    return hipGetLastError();
}

template <int OP, int CT>
static hipError_t launch_wave_ct(const WGeom& g, const StreamArgs& a, hipStream_t s) {
    switch (g.variant) {
        case 0: return launch_wave_t<OP, CT, 13, 3, true>(g, a, s);
        case 1: return launch_wave_t<OP, CT, 3, 2, true>(g, a, s);
        case 2: return launch_wave_t<OP, CT, 13, 2, true>(g, a, s);
        case 3: return launch_wave_t<OP, CT, 7, 1, true>(g, a, s);
        case 4: return launch_wave_t<OP, CT, 4, 4, false>(g, a, s);
        case 5: return launch_wave_t<OP, CT, 8, 4, false>(g, a, s);
        case 6: return launch_wave_t<OP, CT, 16, 2, false>(g, a, s);
        case 7: return launch_wave_t<OP, CT, 16, 3, false>(g, a, s);
        case 8: return launch_wave_t<OP, CT, 16, 4, false>(g, a, s);
        case kTallVariant0 + 0: return launch_wave_t<OP, CT, 8, 2, true, kTallRS>(g, a, s);
        case kTallVariant0 + 1: return launch_wave_t<OP, CT, 8, 2, false, kTallRS>(g, a, s);
        default: return launch_wave_t<OP, CT, 6, 3, false, kTallRS>(g, a, s);
    }
}

template <int OP>
static hipError_t launch_wave_op(const WGeom& g, const StreamArgs& a, hipStream_t s) {
    switch (g.ct) {
        case CT_F32: return launch_wave_ct<OP, CT_F32>(g, a, s);
        case CT_BF16: return launch_wave_ct<OP, CT_BF16>(g, a, s);
        case CT_BF16X2: return launch_wave_ct<OP, CT_BF16X2>(g, a, s);
        default: return launch_wave_ct<OP, CT_BF16X3>(g, a, s);
    }
}

hipError_t launch_wave(int op, const WGeom& g, const StreamArgs& a, hipStream_t s) {
    if (op == OP_SKETCH) return launch_wave_op<OP_SKETCH>(g, a, s);
    if (op == OP_POWER) return launch_wave_op<OP_POWER>(g, a, s);
    return launch_wave_op<OP_TTM>(g, a, s);
}

// Batched instantiations: the generic bounds (row blocks, operand blocks) of
// the short-mode kernel, smallest first, for the compute types of the FP32
// and bf16 paths (the sketch in FP32 or bf16, the other passes in FP32 or
// split bf16).
static const int kBatchShapes[][2] = {{4, 4}, {8, 4}, {16, 2}, {16, 3}, {16, 4}};
constexpr int kNumBatchShapes = 5;

int wave_batch_variant(const WGeom& g) {
    if (g.rs != 1) return -1;
    for (int v = 0; v < kNumBatchShapes; ++v)
        if (g.IB <= kBatchShapes[v][0] && g.NB <= kBatchShapes[v][1]) return v;
    return -1;
}

template <int OP, int CT, int IBT, int NBT>
static hipError_t launch_wave_batch_t(const WaveJob* jobs, int njobs, int max_units, size_t lds,
                                      hipStream_t s) {
    hipLaunchKernelGGL((k_wave_batch<OP, CT, IBT, NBT>), dim3(max_units, njobs), dim3(kBlock), lds, s,
                       jobs);
    return hipGetLastError();
}

template <int OP, int CT>
static hipError_t launch_wave_batch_v(int variant, const WaveJob* jobs, int njobs, int max_units,
                                      size_t lds, hipStream_t s) {
    switch (variant) {
        case 0: return launch_wave_batch_t<OP, CT, 4, 4>(jobs, njobs, max_units, lds, s);
        case 1: return launch_wave_batch_t<OP, CT, 8, 4>(jobs, njobs, max_units, lds, s);
        case 2: return launch_wave_batch_t<OP, CT, 16, 2>(jobs, njobs, max_units, lds, s);
        case 3: return launch_wave_batch_t<OP, CT, 16, 3>(jobs, njobs, max_units, lds, s);
        case 4: return launch_wave_batch_t<OP, CT, 16, 4>(jobs, njobs, max_units, lds, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_wave_batch(int op, int ct, int variant, const WaveJob* jobs, int njobs,
                             int max_units, size_t lds, hipStream_t s) {
    if (njobs < 1 || max_units < 1 || lds + kStaticLdsMargin > kLdsLimit) return hipErrorInvalidValue;
    if (op == OP_SKETCH) {
        if (ct == CT_F32) return launch_wave_batch_v<OP_SKETCH, CT_F32>(variant, jobs, njobs, max_units, lds, s);
        if (ct == CT_BF16) return launch_wave_batch_v<OP_SKETCH, CT_BF16>(variant, jobs, njobs, max_units, lds, s);
    } else if (op == OP_POWER) {
        if (ct == CT_F32) return launch_wave_batch_v<OP_POWER, CT_F32>(variant, jobs, njobs, max_units, lds, s);
        if (ct == CT_BF16X3) return launch_wave_batch_v<OP_POWER, CT_BF16X3>(variant, jobs, njobs, max_units, lds, s);
    } else {
        if (ct == CT_F32) return launch_wave_batch_v<OP_TTM, CT_F32>(variant, jobs, njobs, max_units, lds, s);
        if (ct == CT_BF16X3) return launch_wave_batch_v<OP_TTM, CT_BF16X3>(variant, jobs, njobs, max_units, lds, s);
    }
    return hipErrorInvalidValue;
}

// The compute types that have batched instantiations for a pass.
bool wave_batch_ct(int op, int ct) {
    if (op == OP_SKETCH) return ct == CT_F32 || ct == CT_BF16;
    return ct == CT_F32 || ct == CT_BF16X3;
}

}  // namespace rh
