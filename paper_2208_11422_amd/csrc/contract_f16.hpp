// contract_f16.hpp - spectral contractions with FP16 spectra on matrix cores.
//
// Precision mode "split FP16": the per-frequency PSF spectra are stored once in
// FP16 (each frequency scaled by a power of two so its largest component lies
// in [2^14, 2^15)), which halves the bytes streamed per projection.  The tile
// spectra stay FP32 in HBM and are split on the fly into hi + lo FP16 parts
// (hi = fp16(v), lo = fp16(v - hi)) after a power-of-two scale per (frequency,
// tile) row, so they keep about 22 significant bits; each real product is the
// sum of two FP16 matrix products (hi and lo) accumulated in FP32.  The spectra
// are laid out in MFMA fragment order so that every lane loads one contiguous
// 16- or 32-byte piece.
//
// Fragment layouts (wave64), checked against a CPU product on gfx950:
//   v_mfma_f32_16x16x32_f16: A[i][k] in lane i + 16 (k / 8), element k % 8;
//                            B[k][j] in lane j + 16 (k / 8), element k % 8.
//   v_mfma_f32_16x16x16_f16: A[i][k] in lane i + 16 (k / 4), element k % 4;
//                            B[k][j] in lane j + 16 (k / 4), element k % 4.
//   Both: D[i][j] in lane j + 16 (i / 4), element i % 4.
#pragma once

#include <hip/hip_runtime.h>

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

struct alignas(4) half2c {
    _Float16 re, im;
};

__device__ __forceinline__ f32x4v mfma_h32(f16x8 a, f16x8 b, f32x4v c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4v mfma_h16(f16x4 a, f16x4 b, f32x4v c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
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
__global__ void k_pack_fwd_f16(const float2 *__restrict__ Gf, int KK, int NNp, int nkb,
                               const int *__restrict__ gexp, half2c *__restrict__ Hf, size_t total)
{
    const int ncb = NNp / 16;
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
        half2c h;
        h.re = (_Float16)ldexpf(v.x, ex);
        h.im = (_Float16)ldexpf(v.y, ex);
        Hf[idx] = h;
    }
}

// Adjoint fragments: Hb[k][cc][kb][lane][e], c = 16 cc + 4 (lane / 16) + e,
// kk = 16 kb + lane % 16, value Gb[k][c][kk] 2^gexp[k] (0 past NN or KK).
__global__ void k_pack_adj_f16(const float2 *__restrict__ Gb, int NN, int KK, int ncc, int nkb,
                               const int *__restrict__ gexp, half2c *__restrict__ Hb, size_t total)
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
        half2c h;
        h.re = (_Float16)ldexpf(v.x, ex);
        h.im = (_Float16)ldexpf(v.y, ex);
        Hb[idx] = h;
    }
}

// hi/lo split of a scaled value
__device__ __forceinline__ void split_f16(float v, _Float16 &hi, _Float16 &lo)
{
    hi = (_Float16)v;
    lo = (_Float16)(v - (float)hi);
}

// Forward contraction, split FP16 (see the FP32 k_contract_fwd for the roles):
//   Yp[s][k][t][c] = sum_{kk in chunk} X[k][t][kk] Gf[k][kk][c]
// A = X rows (16 tiles x 32 kk, row stride KKs, scaled by 2^xexp and split),
// B = Hf fragments (32 kk x 16 c), CB blocks of c per wave, U prefetched steps.
// kchunk is a multiple of 32.
template <int CB, int U>
__global__ __launch_bounds__(512) void k_contract_fwd_f16(
    const half2c *__restrict__ Hf, const float2 *__restrict__ X, const unsigned *__restrict__ xmax,
    const int *__restrict__ gexp, float2 *__restrict__ Yp, int NN, int NNp, int KK, int KKs,
    int nkb, int nt, int nf, int kchunk)
{
    const int k = blockIdx.x, s = blockIdx.y, t0 = blockIdx.z * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kg = lane >> 4;
    const int ncb = NNp / 16;
    const int kb0 = s * kchunk;
    const int kb1 = min(KK, kb0 + kchunk);
    const int nsteps = (kb1 - kb0 + 31) / 32;
    const int ngroups = (nsteps + U - 1) / U;
    const int t = min(t0 + col, nt - 1);
    const float2 *xrow = X + ((size_t)k * nt + t) * KKs;
    const int ex = f16_scale_exp(__uint_as_float(xmax[(size_t)k * nt + t]));
    int cbk[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b)
        cbk[b] = min(wave * CB + b, ncb - 1);
    const size_t fbase = (size_t)k * nkb * ncb;
    f32x4v accr[CB], acci[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
        accr[b] = f32x4v{0.f, 0.f, 0.f, 0.f};
        acci[b] = f32x4v{0.f, 0.f, 0.f, 0.f};
    }
    float4 xa0[U][4], xa1[U][4];
    uint4 gb0[U][CB][2], gb1[U][CB][2];
    auto load_group = [&](int grp, float4(&xa)[U][4], uint4(&gb)[U][CB][2]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int step = min(grp * U + u, nsteps - 1);
            const int kk = kb0 + 32 * step + 8 * kg;  // multiple of 8, < KKs
            const float4 *xp = reinterpret_cast<const float4 *>(xrow + kk);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                xa[u][q] = xp[q];
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
    auto compute_group = [&](int grp, const float4(&xa)[U][4], const uint4(&gb)[U][CB][2]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int step = grp * U + u;
            const int kk = kb0 + 32 * step + 8 * kg;
            f16x8 arh, arl, aih, ail;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float4 q = xa[u][e / 2];
                const bool ok = step < nsteps && kk + e < kb1;
                const float re = ok ? ldexpf((e & 1) ? q.z : q.x, ex) : 0.f;
                const float im = ok ? ldexpf((e & 1) ? q.w : q.y, ex) : 0.f;
                _Float16 h, l;
                split_f16(re, h, l);
                arh[e] = h;
                arl[e] = l;
                split_f16(im, h, l);
                aih[e] = h;
                ail[e] = l;
            }
            const f16x8 naih = -aih, nail = -ail;
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const half2c *hp = reinterpret_cast<const half2c *>(&gb[u][b][0]);
                f16x8 gr, gi;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    gr[e] = hp[e].re;
                    gi[e] = hp[e].im;
                }
                accr[b] = mfma_h32(arh, gr, accr[b]);
                accr[b] = mfma_h32(arl, gr, accr[b]);
                accr[b] = mfma_h32(naih, gi, accr[b]);
                accr[b] = mfma_h32(nail, gi, accr[b]);
                acci[b] = mfma_h32(arh, gi, acci[b]);
                acci[b] = mfma_h32(arl, gi, acci[b]);
                acci[b] = mfma_h32(aih, gr, acci[b]);
                acci[b] = mfma_h32(ail, gr, acci[b]);
            }
        }
    };
    if (ngroups > 0)
        load_group(0, xa0, gb0);
    for (int grp = 0; grp < ngroups; grp += 2) {
        if (grp + 1 < ngroups)
            load_group(grp + 1, xa1, gb1);
        compute_group(grp, xa0, gb0);
        if (grp + 1 < ngroups) {
            if (grp + 2 < ngroups)
                load_group(grp + 2, xa0, gb0);
            compute_group(grp + 1, xa1, gb1);
        }
    }
    // D[t][c] rows t0 + 4 kg + i carry the scale 2^(xexp[row] + gexp[k])
    float2 *yk = Yp + ((size_t)s * nf + k) * nt * NN;
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
            if (c < NN)
                yk[(size_t)tt * NN + c] = make_float2(ldexpf(accr[b][i], sc), ldexpf(acci[b][i], sc));
        }
    }
}

// Adjoint contraction, split FP16:
//   B[k][t][kk] = sum_c R[k][t][c] conj(Gb[k][c][kk])
// A = R rows (16 tiles x 16 c per step, scaled by 2^rexp and split hi/lo once
// per block into LDS), B = Hb fragments (16 c x 16 kk), CB blocks of kk per
// wave, U prefetched steps.
template <int CB, int U>
__global__ __launch_bounds__(256) void k_contract_adj_f16(
    const half2c *__restrict__ Hb, const float2 *__restrict__ Rs, const unsigned *__restrict__ rmax,
    const int *__restrict__ gexp, float2 *__restrict__ B, int NN, int NNp, int KK, int nkb,
    int nt)
{
    // LDS: per 16-c chunk and lane, 4 c values x {re hi, re lo, im hi, im lo}
    extern __shared__ _Float16 ra[];
    const int k = blockIdx.x, t0 = blockIdx.z * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int col = lane & 15, kg = lane >> 4;
    const int ncc = NNp / 16;
    for (int idx = threadIdx.x; idx < ncc * 64 * 4; idx += blockDim.x) {
        const int e = idx % 4, l = (idx / 4) % 64, cc = idx / 256;
        const int c = 16 * cc + 4 * (l / 16) + e;
        const int tt = t0 + l % 16;
        float2 v = make_float2(0.f, 0.f);
        int ex = 0;
        if (c < NN && tt < nt) {
            v = Rs[((size_t)k * nt + tt) * NN + c];
            ex = f16_scale_exp(__uint_as_float(rmax[(size_t)k * nt + tt]));
        }
        _Float16 h, lo;
        _Float16 *dst = ra + ((size_t)(cc * 64 + l) * 4 + e) * 4;
        split_f16(ldexpf(v.x, ex), h, lo);
        dst[0] = h;
        dst[1] = lo;
        split_f16(ldexpf(v.y, ex), h, lo);
        dst[2] = h;
        dst[3] = lo;
    }
    __syncthreads();
    int kbk[CB];
    bool k_ok[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
        const int kb = (blockIdx.y * nwaves + wave) * CB + b;
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
    const int ngroups = (ncc + U - 1) / U;
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
            if (cc >= ncc)
                break;
            const _Float16 *src = ra + (size_t)(cc * 64 + lane) * 16;
            f16x4 rrh, rrl, rih, ril;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                rrh[e] = src[4 * e + 0];
                rrl[e] = src[4 * e + 1];
                rih[e] = src[4 * e + 2];
                ril[e] = src[4 * e + 3];
            }
            const f16x4 nrrh = -rrh, nrrl = -rrl;
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const half2c *hp = reinterpret_cast<const half2c *>(&gb[u][b]);
                f16x4 gr, gi;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    gr[e] = hp[e].re;
                    gi[e] = hp[e].im;
                }
                // conj(G) R = (Gr Rr + Gi Ri) + i (Gr Ri - Gi Rr)
                accr[b] = mfma_h16(rrh, gr, accr[b]);
                accr[b] = mfma_h16(rrl, gr, accr[b]);
                accr[b] = mfma_h16(rih, gi, accr[b]);
                accr[b] = mfma_h16(ril, gi, accr[b]);
                acci[b] = mfma_h16(rih, gr, acci[b]);
                acci[b] = mfma_h16(ril, gr, acci[b]);
                acci[b] = mfma_h16(nrrh, gi, acci[b]);
                acci[b] = mfma_h16(nrrl, gi, acci[b]);
            }
        }
    };
    if (ngroups > 0)
        load_group(0, gb0);
    for (int grp = 0; grp < ngroups; grp += 2) {
        if (grp + 1 < ngroups)
            load_group(grp + 1, gb1);
        compute_group(grp, gb0);
        if (grp + 1 < ngroups) {
            if (grp + 2 < ngroups)
                load_group(grp + 2, gb0);
            compute_group(grp + 1, gb1);
        }
    }
    float2 *bk = B + (size_t)k * nt * KK;
    const int gx = gexp[k];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int tt = t0 + 4 * kg + i;
        if (tt >= nt)
            continue;
        const int sc = -(f16_scale_exp(__uint_as_float(rmax[(size_t)k * nt + tt])) + gx);
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const int kk = 16 * kbk[b] + col;
            if (k_ok[b] && kk < KK)
                bk[(size_t)tt * KK + kk] = make_float2(ldexpf(accr[b][i], sc), ldexpf(acci[b][i], sc));
        }
    }
}
