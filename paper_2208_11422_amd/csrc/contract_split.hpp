// contract_split.hpp - spectral contractions with 16-bit spectra on matrix cores.
//
// Split precision modes (FP16 or BF16 storage): the per-frequency PSF spectra
// are stored once in the 16-bit type (each frequency scaled by a power of two
// so its largest component lies in [2^14, 2^15)), which halves the bytes
// streamed per projection.  The tile spectra stay FP32 in HBM and are split on
// the fly into hi + lo parts (hi = round(v), lo = round(v - hi)) after a
// power-of-two scale per (frequency, tile) row; each real product is the sum
// of two 16-bit matrix products (hi and lo) accumulated in FP32.  FP16 keeps
// 11 significant bits per spectrum value and about 22 per tile value; BF16
// keeps 8 and about 16.  The spectra are laid out in MFMA fragment order so
// that every lane loads one contiguous 16- or 32-byte piece.
//
// Fragment layouts (wave64), checked against a CPU product on gfx950 for
// both types:
//   16x16x32: A[i][k] in lane i + 16 (k / 8), element k % 8;
//             B[k][j] in lane j + 16 (k / 8), element k % 8.
//   16x16x16: A[i][k] in lane i + 16 (k / 4), element k % 4;
//             B[k][j] in lane j + 16 (k / 4), element k % 4.
//   Both: D[i][j] in lane j + 16 (i / 4), element i % 4.
#pragma once

#include <hip/hip_runtime.h>

typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

// one complex spectrum value in a 16-bit type
template <typename S>
struct alignas(4) cplx16 {
    S re, im;
};

struct PrecF16 {
    typedef _Float16 S;
    typedef _Float16 v8 __attribute__((ext_vector_type(8)));
    typedef _Float16 v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ S from(float v) { return (S)v; }
    static __device__ __forceinline__ float to(S s) { return (float)s; }
    static __device__ __forceinline__ f32x4v m32(v8 a, v8 b, f32x4v c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ f32x4v m16(v4 a, v4 b, f32x4v c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    }
};

struct PrecBF16 {
    typedef __bf16 S;
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
    typedef __bf16 v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ S from(float v) { return (S)v; }
    static __device__ __forceinline__ float to(S s) { return (float)s; }
    static __device__ __forceinline__ f32x4v m32(v8 a, v8 b, f32x4v c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ f32x4v m16(v4 a, v4 b, f32x4v c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a),
                                                         __builtin_bit_cast(s16x4, b), c, 0, 0,
                                                         0);
    }
};

// sign flip of every element (exact for both types)
template <typename V, typename U>
__device__ __forceinline__ V neg16(V v)
{
    return __builtin_bit_cast(V, __builtin_bit_cast(U, v) ^ (unsigned short)0x8000);
}

// Exponent e with max * 2^e in [2^14, 2^15) (0 for max == 0 or not finite).
__device__ __forceinline__ int f16_scale_exp(float m)
{
    if (!(m > 0.f) || !(m < 3.0e38f))
        return 0;
    int e;
    frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
    return 15 - e;
}

// Per-frequency exponent of the spectra: gexp[k] from the largest |re| or |im|
// of Gf[k] (per_k complex values).  One block per frequency.
__global__ void k_spec_exp(const float2 *__restrict__ Gf, size_t per_k, int *__restrict__ gexp)
{
    __shared__ float red[256];
    const float2 *g = Gf + blockIdx.x * per_k;
    float m = 0.f;
    for (size_t i = threadIdx.x; i < per_k; i += blockDim.x)
        m = fmaxf(m, fmaxf(fabsf(g[i].x), fabsf(g[i].y)));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        gexp[blockIdx.x] = f16_scale_exp(red[0]);
}

// Forward fragments: Hf[k][kb][cb][lane][e], kk = 32 kb + 8 (lane / 16) + e,
// c = 16 cb + lane % 16, value Gf[k][kk][c] 2^gexp[k] (0 past KK).
template <class P>
__global__ void k_pack_fwd_split(const float2 *__restrict__ Gf, int KK, int NNp, int ncb, int nkb,
                                 const int *__restrict__ gexp,
                                 cplx16<typename P::S> *__restrict__ Hf, size_t total)
{
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int e = idx % 8;
        const int lane = (idx / 8) % 64;
        const size_t frag = idx / 512;
        const int cb = frag % ncb;
        const size_t kb = (frag / ncb) % nkb;
        const size_t k = frag / ((size_t)ncb * nkb);
        const int kk = (int)(32 * kb) + 8 * (lane / 16) + e;
        const int c = 16 * cb + lane % 16;
        float2 v = make_float2(0.f, 0.f);
        if (kk < KK)
            v = Gf[(k * KK + kk) * NNp + c];
        const int ex = gexp[k];
        cplx16<typename P::S> h;
        h.re = P::from(ldexpf(v.x, ex));
        h.im = P::from(ldexpf(v.y, ex));
        Hf[idx] = h;
    }
}

// Adjoint fragments: Hb[k][cc][kb][lane][e], c = 16 cc + 4 (lane / 16) + e,
// kk = 16 kb + lane % 16, value Gb[k][c][kk] 2^gexp[k] (0 past NN or KK).
template <class P>
__global__ void k_pack_adj_split(const float2 *__restrict__ Gb, int NN, int KK, int ncc, int nkb,
                                 const int *__restrict__ gexp,
                                 cplx16<typename P::S> *__restrict__ Hb, size_t total)
{
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int e = idx % 4;
        const int lane = (idx / 4) % 64;
        const size_t frag = idx / 256;
        const size_t kb = frag % nkb;
        const int cc = (frag / nkb) % ncc;
        const size_t k = frag / ((size_t)nkb * ncc);
        const int c = 16 * cc + 4 * (lane / 16) + e;
        const int kk = (int)(16 * kb) + lane % 16;
        float2 v = make_float2(0.f, 0.f);
        if (c < NN && kk < KK)
            v = Gb[(k * NN + c) * KK + kk];
        const int ex = gexp[k];
        cplx16<typename P::S> h;
        h.re = P::from(ldexpf(v.x, ex));
        h.im = P::from(ldexpf(v.y, ex));
        Hb[idx] = h;
    }
}

// hi/lo split of a scaled value
template <class P>
__device__ __forceinline__ void split_lohi(float v, typename P::S &hi, typename P::S &lo)
{
    hi = P::from(v);
    lo = P::from(v - P::to(hi));
}

// Forward contraction, split precision (see the FP32 k_contract_fwd for the
// roles):
//   Yp[s][k][t][c] = sum_{kk in chunk} X[k][t][kk] Gf[k][kk][c]
// A = X rows (16 tiles x 32 kk per step, row stride KKs, scaled by 2^xexp and
// split hi/lo), B = Hf fragments (32 kk x 16 c), CB blocks of c per wave, U
// steps per group.  Every wave needs the same A fragments, so the block
// converts them once per group into a double-buffered LDS buffer (element
// (L, e) of lane L's eight kk by thread tid + m * blockDim, the same element
// in every group), one barrier per group; the B fragments are prefetched one
// group ahead per wave (clamped loads; surplus steps meet zero A).  kchunk is
// a multiple of 32.  The lone output column xcol (if any) is summed in FP32
// by the converting threads from the values they load, then per tile in a
// fixed order.
template <class P, int CB, int U>
__global__ __launch_bounds__(512) void k_contract_fwd_split(
    const cplx16<typename P::S> *__restrict__ Hf, const float2 *__restrict__ X,
    const unsigned *__restrict__ xmax, const int *__restrict__ gexp, float2 *__restrict__ Yp,
    int NN, int NNp, int KK, int KKs, int nkb, int nt, int nf, int kchunk,
    const int *__restrict__ skip, FreqMap fm, const float2 *__restrict__ Gx, int xcol)
// (xmax: nf * nt maxima, see k_rowmax_reduce)
{
    if (skip && *skip)
        return;
    typedef typename P::S S;
    typedef typename P::v8 V8;
    // A fragments: [buffer][step][lane][re hi, re lo, im hi, im lo], 8 values each
    __shared__ uint4 la[2][U][64][4];
    constexpr int kElems = 512 * U;  // (step, lane, element) per group
    constexpr int KS = (kElems + 319) / 320;  // slots per thread (blocks of >= 320 threads)
    __shared__ float2 colred[kElems];
    int k, s, tg;
    contraction_block(k, s, tg);
    k = unique_freq(k, fm);
    const int t0 = tg * 16;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, kg = lane >> 4;
    const int ncb = NNp / 16;
    const int kb0 = s * kchunk;
    const int kb1 = min(KK, kb0 + kchunk);
    const int nsteps = (kb1 - kb0 + 31) / 32;
    const int ngroups = (nsteps + U - 1) / U;
    int cbk[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b)
        cbk[b] = min(wave * CB + b, ncb - 1);
    const size_t fbase = (size_t)k * nkb * ncb;
    // waves past the column blocks (a block has at least 5 waves for the
    // conversion slots) only convert
    const bool cwave = wave * CB < ncb;
    f32x4v accr[CB], acci[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
        accr[b] = f32x4v{0.f, 0.f, 0.f, 0.f};
        acci[b] = f32x4v{0.f, 0.f, 0.f, 0.f};
    }
    // this thread's conversion slots: element idx = tid + m * nthr of a group
    // (step u = idx / 512, lane L = idx / 8 % 64, element e = idx % 8: tile
    // t0 + L % 16, kk = 32 step + 8 (L / 16) + e)
    const float2 *xs[KS];
    int xe[KS];
    bool live[KS];
#pragma unroll
    for (int m = 0; m < KS; ++m) {
        const int idx = tid + m * nthr;
        live[m] = idx < kElems;
        const int L = (idx >> 3) & 63;
        const int tt = min(t0 + (L & 15), nt - 1);
        xs[m] = X + ((size_t)k * nt + tt) * KKs + kb0 + 8 * (L >> 4) + (idx & 7);
        xe[m] = f16_scale_exp(__uint_as_float(xmax[(size_t)k * nt + tt]));
    }
    const float2 *gxk = Gx + (xcol >= 0 ? (size_t)k * KKs + kb0 : 0);
    float2 xv[KS], gv[KS], accx[KS];
#pragma unroll
    for (int m = 0; m < KS; ++m)
        accx[m] = make_float2(0.f, 0.f);
    auto a_load = [&](int grp) {
#pragma unroll
        for (int m = 0; m < KS; ++m) {
            if (!live[m])
                continue;
            const int idx = tid + m * nthr;
            const int step = min(grp * U + idx / 512, nsteps - 1);
            xv[m] = xs[m][32 * step];
            if (xcol >= 0)
                gv[m] = gxk[32 * step + 8 * (((idx >> 3) & 63) >> 4) + (idx & 7)];
        }
    };
    auto a_store = [&](int grp, int buf) {
#pragma unroll
        for (int m = 0; m < KS; ++m) {
            if (!live[m])
                continue;
            const int idx = tid + m * nthr;
            const int u = idx / 512, L = (idx >> 3) & 63, e = idx & 7;
            const int step = grp * U + u;
            const int kk = kb0 + 32 * step + 8 * (L >> 4) + e;
            const bool ok = step < nsteps && kk < kb1;
            const float re = ok ? xv[m].x : 0.f, im = ok ? xv[m].y : 0.f;
            S h, l;
            S *dst = reinterpret_cast<S *>(&la[buf][u][L][0]);
            split_lohi<P>(ldexpf(re, xe[m]), h, l);
            dst[e] = h;
            dst[8 + e] = l;
            split_lohi<P>(ldexpf(im, xe[m]), h, l);
            dst[16 + e] = h;
            dst[24 + e] = l;
            if (xcol >= 0) {
                accx[m].x = fmaf(re, gv[m].x, fmaf(-im, gv[m].y, accx[m].x));
                accx[m].y = fmaf(re, gv[m].y, fmaf(im, gv[m].x, accx[m].y));
            }
        }
    };
    uint4 gb0[U][CB][2], gb1[U][CB][2];
    auto b_load = [&](int grp, uint4(&gb)[U][CB][2]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int step = min(grp * U + u, nsteps - 1);
            const size_t kbi = (size_t)(kb0 / 32 + step);
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const uint4 *gp = reinterpret_cast<const uint4 *>(
                    Hf + ((fbase + kbi * ncb + cbk[b]) * 64 + lane) * 8);
                gb[u][b][0] = gp[0];
                gb[u][b][1] = gp[1];
            }
        }
    };
    auto compute_group = [&](int buf, const uint4(&gb)[U][CB][2]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint4 q0 = la[buf][u][lane][0], q1 = la[buf][u][lane][1];
            const uint4 q2 = la[buf][u][lane][2], q3 = la[buf][u][lane][3];
            const V8 arh = *reinterpret_cast<const V8 *>(&q0), arl = *reinterpret_cast<const V8 *>(&q1);
            const V8 aih = *reinterpret_cast<const V8 *>(&q2), ail = *reinterpret_cast<const V8 *>(&q3);
            const V8 naih = neg16<V8, u16x8>(aih), nail = neg16<V8, u16x8>(ail);
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const cplx16<S> *hp = reinterpret_cast<const cplx16<S> *>(&gb[u][b][0]);
                V8 gr, gi;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    gr[e] = hp[e].re;
                    gi[e] = hp[e].im;
                }
                accr[b] = P::m32(arh, gr, accr[b]);
                accr[b] = P::m32(arl, gr, accr[b]);
                accr[b] = P::m32(naih, gi, accr[b]);
                accr[b] = P::m32(nail, gi, accr[b]);
                acci[b] = P::m32(arh, gi, acci[b]);
                acci[b] = P::m32(arl, gi, acci[b]);
                acci[b] = P::m32(aih, gr, acci[b]);
                acci[b] = P::m32(ail, gr, acci[b]);
            }
        }
    };
    a_load(0);
    if (cwave)
        b_load(0, gb0);
    a_store(0, 0);
    __syncthreads();
    for (int grp = 0; grp < ngroups; grp += 2) {
        a_load(grp + 1);
        if (cwave) {
            b_load(grp + 1, gb1);
            compute_group(0, gb0);
        }
        a_store(grp + 1, 1);
        __syncthreads();
        a_load(grp + 2);
        if (cwave) {
            b_load(grp + 2, gb0);
            compute_group(1, gb1);
        }
        a_store(grp + 2, 0);
        __syncthreads();
    }
    // D[t][c] rows t0 + 4 kg + i carry the scale 2^(xexp[row] + gexp[k])
    float2 *yk = Yp + ((size_t)s * nf + k) * nt * NN;
    if (xcol >= 0) {
        // lone column: the slots' partial sums per tile, in element order
#pragma unroll
        for (int m = 0; m < KS; ++m)
            if (live[m])
                colred[tid + m * nthr] = accx[m];
        __syncthreads();
        if (tid < 16 && t0 + tid < nt) {
            float2 a = make_float2(0.f, 0.f);
            for (int u = 0; u < U; ++u)
                for (int q = 0; q < 4; ++q)
                    for (int e = 0; e < 8; ++e) {
                        const float2 v = colred[u * 512 + (q * 16 + tid) * 8 + e];
                        a.x += v.x;
                        a.y += v.y;
                    }
            yk[(size_t)(t0 + tid) * NN + xcol] = a;
        }
    }
    const int gx = gexp[k];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int tt = t0 + 4 * kg + i;
        if (tt >= nt)
            continue;
        const int sc = -(f16_scale_exp(__uint_as_float(xmax[(size_t)k * nt + tt])) + gx);
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const int c = 16 * (wave * CB + b) + col;
            if (c < NN && wave * CB + b < ncb)
                yk[(size_t)tt * NN + c] = make_float2(ldexpf(accr[b][i], sc), ldexpf(acci[b][i], sc));
        }
    }
}

// Rows (16-c chunks) of image tile spectra the split adjoint stages in LDS:
// whole register groups of U chunks, zero past the ncc fragment chunks.
__host__ __device__ __forceinline__ int split_adj_chunks(int ncc, int U)
{
    return (ncc + U - 1) / U * U;
}

// Adjoint contraction, split precision:
//   B[k][t][kk] = sum_c R[k][t][c] conj(Gb[k][c][kk])
// A = R rows (16 tiles x 16 c per step, scaled by 2^rexp and split hi/lo once
// per block into LDS, zero past NN), B = Hb fragments (16 c x 16 kk), CB
// blocks of kk per wave, U prefetched steps in a straight-line
// double-buffered loop (an odd last group has no partner; chunks past ncc
// meet zeros in LDS).  A block covers `ranges` kk ranges from one staging of
// R; three blocks per CU are asked of the register allocator (the loop over
// ranges otherwise costs one: measured 0.636 against 0.696 ms).
template <class P, int CB, int U>
__global__ __launch_bounds__(256, 3) void k_contract_adj_split(
    const cplx16<typename P::S> *__restrict__ Hb, const float2 *__restrict__ Rs,
    const unsigned *__restrict__ rmax, const int *__restrict__ gexp, float2 *__restrict__ B,
    int NN, int NNp, int KK, int KKs, int nkb, int nt, const int *__restrict__ skip, FreqMap fm,
    const float2 *__restrict__ Hx, int xc, int KKb, size_t osk, size_t ost, int ranges)
{
    if (skip && *skip)
        return;
    typedef typename P::S S;
    typedef typename P::v4 V4;
    // LDS: per 16-c chunk and lane, 4 c values x {re hi, re lo, im hi, im lo}
    extern __shared__ unsigned short ra_bits[];
    S *ra = reinterpret_cast<S *>(ra_bits);
    int k, by, tg;
    contraction_block(k, by, tg);
    k = unique_freq(k, fm);
    const int t0 = tg * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int col = lane & 15, kg = lane >> 4;
    const int ncc = NNp / 16;
    const int ncl = split_adj_chunks(ncc, U);
    for (int idx = threadIdx.x; idx < ncl * 64 * 4; idx += blockDim.x) {
        const int e = idx % 4, l = (idx / 4) % 64, cc = idx / 256;
        const int c = 16 * cc + 4 * (l / 16) + e;
        const int tt = t0 + l % 16;
        float2 v = make_float2(0.f, 0.f);
        int ex = 0;
        if (c < NN && c < 16 * ncc && tt < nt) {
            v = Rs[((size_t)k * nt + tt) * NN + c];
            ex = f16_scale_exp(__uint_as_float(rmax[(size_t)k * nt + tt]));
        }
        S h, lo;
        S *dst = ra + ((size_t)(cc * 64 + l) * 4 + e) * 4;
        split_lohi<P>(ldexpf(v.x, ex), h, lo);
        dst[0] = h;
        dst[1] = lo;
        split_lohi<P>(ldexpf(v.y, ex), h, lo);
        dst[2] = h;
        dst[3] = lo;
    }
    __syncthreads();
    // `ranges` kk ranges per block, all from the R staged once above
    for (int rg = 0; rg < ranges; ++rg) {
        const int kbw = ((by * ranges + rg) * nwaves + wave) * CB;
        if (kbw >= nkb)
            break;  // (wave-uniform; no barriers below)
        int kbk[CB];
        bool k_ok[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const int kb = kbw + b;
            k_ok[b] = kb < nkb;
            kbk[b] = min(kb, nkb - 1);
        }
        f32x4v accr[CB], acci[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            accr[b] = f32x4v{0.f, 0.f, 0.f, 0.f};
            acci[b] = f32x4v{0.f, 0.f, 0.f, 0.f};
        }
        const size_t fbase = (size_t)k * ncc * nkb;
        const int ngroups = ncl / U;
        uint4 gb0[U][CB], gb1[U][CB];
        auto load_group = [&](int grp, uint4(&gb)[U][CB]) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int cc = min(grp * U + u, ncc - 1);
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    gb[u][b] = *reinterpret_cast<const uint4 *>(
                        Hb + ((fbase + (size_t)cc * nkb + kbk[b]) * 64 + lane) * 4);
            }
        };
        auto compute_group = [&](int grp, const uint4(&gb)[U][CB]) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int cc = grp * U + u;
                const S *src = ra + (size_t)(cc * 64 + lane) * 16;
                V4 rrh, rrl, rih, ril;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    rrh[e] = src[4 * e + 0];
                    rrl[e] = src[4 * e + 1];
                    rih[e] = src[4 * e + 2];
                    ril[e] = src[4 * e + 3];
                }
                const V4 nrrh = neg16<V4, u16x4>(rrh), nrrl = neg16<V4, u16x4>(rrl);
                V4 gr[CB], gi[CB];
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    const cplx16<S> *hp = reinterpret_cast<const cplx16<S> *>(&gb[u][b]);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        gr[b][e] = hp[e].re;
                        gi[b][e] = hp[e].im;
                    }
                }
                // conj(G) R = (Gr Rr + Gi Ri) + i (Gr Ri - Gi Rr), product-major
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    accr[b] = P::m16(rrh, gr[b], accr[b]);
                    acci[b] = P::m16(rih, gr[b], acci[b]);
                }
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    accr[b] = P::m16(rrl, gr[b], accr[b]);
                    acci[b] = P::m16(ril, gr[b], acci[b]);
                }
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    accr[b] = P::m16(rih, gi[b], accr[b]);
                    acci[b] = P::m16(nrrh, gi[b], acci[b]);
                }
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    accr[b] = P::m16(ril, gi[b], accr[b]);
                    acci[b] = P::m16(nrrl, gi[b], acci[b]);
                }
            }
        };
        load_group(0, gb0);
        for (int grp = 0; grp < ngroups; grp += 2) {
            load_group(grp + 1, gb1);
            __builtin_amdgcn_sched_barrier(0);
            compute_group(grp, gb0);
            __builtin_amdgcn_sched_barrier(0);
            load_group(grp + 2, gb0);
            __builtin_amdgcn_sched_barrier(0);
            if (grp + 1 < ngroups)  // an odd last group has no partner
                compute_group(grp + 1, gb1);
            __builtin_amdgcn_sched_barrier(0);
        }
        float2 *bk = B + (size_t)k * osk;   // rows of KKs: 128-byte aligned
        const int gx = gexp[k];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int tt = t0 + 4 * kg + i;
            if (tt >= nt)
                continue;
            const int sc = -(f16_scale_exp(__uint_as_float(rmax[(size_t)k * nt + tt])) + gx);
            // the lone reduction index xc (if any), in float32: + R[t][xc] conj(H[xc][kk])
            const float2 r = xc >= 0 ? Rs[((size_t)k * nt + tt) * NN + xc] : make_float2(0.f, 0.f);
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const int kk = 16 * kbk[b] + col;
                float2 o = make_float2(ldexpf(accr[b][i], sc), ldexpf(acci[b][i], sc));
                if (xc >= 0) {
                    const float2 h = Hx[(size_t)k * KKb + 16 * kbk[b] + col];
                    o.x = fmaf(r.x, h.x, fmaf(r.y, h.y, o.x));
                    o.y = fmaf(r.y, h.x, fmaf(-r.x, h.y, o.y));
                }
                if (k_ok[b] && kk < KK)
                    bk[(size_t)tt * ost + kk] = o;
            }
        }
    }
}
