// tile_fft.hpp - Q x Q tile DFTs as mixed-radix FFTs held in registers.
//
// One thread transforms one length-Q sequence (or two real sequences packed
// as one complex one) entirely in registers.  Q is a template parameter, so
// every radix stage is unrolled with compile-time indices; twiddles
// exp(2 pi i m / Q) come from a Q-entry table read with uniform (scalar)
// loads.  Stages follow the Stockham autosort ordering (each radix-R stage
// multiplies by exp(-+2 pi i k r / (Ns R)) and writes its outputs Ns apart),
// so no digit reversal is needed.  Tiles live in LDS between the row pass
// and the column pass, exactly as in the direct-sum kernels they replace.
#pragma once

#include <hip/hip_runtime.h>

namespace tfft {

template <int L>
constexpr int radix_of()
{
    return (L % 4 == 0 && L != 8) ? 4 : (L % 2 == 0) ? 2 : (L % 3 == 0) ? 3 : (L % 5 == 0) ? 5
                                                         : (L % 7 == 0) ? 7 : L;
}

// cos and sin of 2 pi m / Q as compile-time constants: Taylor series in double
// of the angle reduced to (-pi, pi], rounded once to float.  Inside the
// unrolled transforms m is a constant, so a twiddle is an immediate operand
// rather than a table load.
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double taylor_cos(double x)
{
    double t = 1.0, s = 1.0;
    for (int n = 1; n <= 30; ++n) {
        t *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
        s += t;
    }
    return s;
}
constexpr double taylor_sin(double x)
{
    double t = x, s = x;
    for (int n = 1; n <= 30; ++n) {
        t *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
        s += t;
    }
    return s;
}
template <int Q>
struct TwTable {
    float c[Q], s[Q];
    constexpr TwTable() : c(), s()
    {
        for (int m = 0; m < Q; ++m) {
            const int mm = 2 * m > Q ? m - Q : m;
            const double a = kTwoPi * mm / Q;
            c[m] = (float)taylor_cos(a);
            s[m] = (float)taylor_sin(a);
        }
    }
};

// exp(SIGN * 2 pi i m / Q), m a compile-time constant after unrolling
template <int Q, int SIGN>
__device__ __forceinline__ float2 twid_c(int m)
{
    constexpr TwTable<Q> t{};
    return make_float2(t.c[m], SIGN > 0 ? t.s[m] : -t.s[m]);
}

// exp(SIGN * 2 pi i m / n) from a table tw[m] = (cos, sin)(2 pi m / n) (for
// transforms whose length is known only at run time)
template <int SIGN>
__device__ __forceinline__ float2 twid(const float2 *__restrict__ tw, int m)
{
    const float2 t = tw[m];
    return SIGN > 0 ? t : make_float2(t.x, -t.y);
}

__device__ __forceinline__ float2 cmulf(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// cos and sin of 2 pi m / R for the odd radices (float constants; the tables
// are exactly symmetric: cos(m) = cos(R - m), sin(m) = -sin(R - m))
template <int R>
__device__ __forceinline__ float root_cos(int m)
{
    if constexpr (R == 3) {
        constexpr float t[3] = {1.0f, -0.5f, -0.5f};
        return t[m];
    } else if constexpr (R == 5) {
        constexpr float t[5] = {1.0f, 0.30901699437494745f, -0.8090169943749475f,
                                -0.8090169943749475f, 0.30901699437494745f};
        return t[m];
    } else {
        constexpr float t[7] = {1.0f, 0.6234898018587336f, -0.22252093395631440f,
                                -0.9009688679024191f, -0.9009688679024191f,
                                -0.22252093395631440f, 0.6234898018587336f};
        return t[m];
    }
}

template <int R>
__device__ __forceinline__ float root_sin(int m)
{
    if constexpr (R == 3) {
        constexpr float t[3] = {0.0f, 0.8660254037844386f, -0.8660254037844386f};
        return t[m];
    } else if constexpr (R == 5) {
        constexpr float t[5] = {0.0f, 0.9510565162951535f, 0.5877852522924731f,
                                -0.5877852522924731f, -0.9510565162951535f};
        return t[m];
    } else {
        constexpr float t[7] = {0.0f, 0.7818314824680298f, 0.9749279121818236f,
                                0.4338837391175582f, -0.4338837391175582f,
                                -0.9749279121818236f, -0.7818314824680298f};
        return t[m];
    }
}

// Odd R-point DFT (R = 3, 5, 7) from the pairs q, R - q: with a_q = v[q] +
// v[R-q] and b_q = v[q] - v[R-q],
//   X[k], X[R-k] = v[0] + sum_q cos(2 pi q k / R) a_q  +- SIGN i sum_q sin(2 pi q k / R) b_q,
// about a third of the multiplies of the direct sum.
template <int R, int SIGN>
__device__ __forceinline__ void dft_odd(float2 (&v)[R])
{
    constexpr int H = (R - 1) / 2;
    float2 a[H], b[H];
    float2 sum = v[0];
#pragma unroll
    for (int q = 1; q <= H; ++q) {
        a[q - 1] = make_float2(v[q].x + v[R - q].x, v[q].y + v[R - q].y);
        b[q - 1] = make_float2(v[q].x - v[R - q].x, v[q].y - v[R - q].y);
        sum.x += a[q - 1].x;
        sum.y += a[q - 1].y;
    }
    float2 o[R];
    o[0] = sum;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        float2 c = v[0], s = make_float2(0.f, 0.f);
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            const float cq = root_cos<R>((q * k) % R), sq = root_sin<R>((q * k) % R);
            c.x = fmaf(cq, a[q - 1].x, c.x);
            c.y = fmaf(cq, a[q - 1].y, c.y);
            s.x = fmaf(sq, b[q - 1].x, s.x);
            s.y = fmaf(sq, b[q - 1].y, s.y);
        }
        // SIGN i s = SIGN (-s.y, s.x)
        const float isx = SIGN > 0 ? -s.y : s.y, isy = SIGN > 0 ? s.x : -s.x;
        o[k] = make_float2(c.x + isx, c.y + isy);
        o[R - k] = make_float2(c.x - isx, c.y - isy);
    }
#pragma unroll
    for (int p = 0; p < R; ++p)
        v[p] = o[p];
}

// In-place R-point DFT, natural order: v[p] <- sum_q v[q] exp(SIGN 2 pi i p q / R).
template <int R, int SIGN, int Q>
__device__ __forceinline__ void dft_small(float2 (&v)[R], const float2 *__restrict__ tw)
{
    if constexpr (R == 2) {
        const float2 a = v[0], b = v[1];
        v[0] = make_float2(a.x + b.x, a.y + b.y);
        v[1] = make_float2(a.x - b.x, a.y - b.y);
    } else if constexpr (R == 4) {
        const float2 a = v[0], b = v[1], c = v[2], d = v[3];
        const float2 s0 = make_float2(a.x + c.x, a.y + c.y), s1 = make_float2(a.x - c.x, a.y - c.y);
        const float2 s2 = make_float2(b.x + d.x, b.y + d.y), s3 = make_float2(b.x - d.x, b.y - d.y);
        // s3 * (SIGN i)
        const float2 s3r = SIGN > 0 ? make_float2(-s3.y, s3.x) : make_float2(s3.y, -s3.x);
        v[0] = make_float2(s0.x + s2.x, s0.y + s2.y);
        v[2] = make_float2(s0.x - s2.x, s0.y - s2.y);
        v[1] = make_float2(s1.x + s3r.x, s1.y + s3r.y);
        v[3] = make_float2(s1.x - s3r.x, s1.y - s3r.y);
    } else if constexpr (R == 3 || R == 5 || R == 7) {
        dft_odd<R, SIGN>(v);
    } else {
        float2 o[R];
#pragma unroll
        for (int p = 0; p < R; ++p) {
            float2 acc = v[0];
#pragma unroll
            for (int q = 1; q < R; ++q) {
                const float2 w = twid_c<Q, SIGN>(((p * q) % R) * (Q / R));
                acc.x = fmaf(v[q].x, w.x, fmaf(-v[q].y, w.y, acc.x));
                acc.y = fmaf(v[q].x, w.y, fmaf(v[q].y, w.x, acc.y));
            }
            o[p] = acc;
        }
#pragma unroll
        for (int p = 0; p < R; ++p)
            v[p] = o[p];
    }
}

// One Stockham stage of radix R with span Ns: in -> out.
template <int Q, int R, int Ns, int SIGN>
__device__ __forceinline__ void stage(const float2 (&in)[Q], float2 (&out)[Q],
                                      const float2 *__restrict__ tw)
{
#pragma unroll
    for (int j = 0; j < Q / R; ++j) {
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            v[r] = in[j + r * (Q / R)];
        const int k = j % Ns;
        if (k != 0) {
#pragma unroll
            for (int r = 1; r < R; ++r)
                v[r] = cmulf(v[r], twid_c<Q, SIGN>((k * r * (Q / (Ns * R))) % Q));
        }
        dft_small<R, SIGN, Q>(v, tw);
        const int base = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r)
            out[base + r * Ns] = v[r];
    }
}

template <int Q, int Ns, int SIGN>
__device__ __forceinline__ void stages(float2 (&a)[Q], float2 (&b)[Q], const float2 *__restrict__ tw)
{
    if constexpr (Ns < Q) {
        constexpr int R = radix_of<Q / Ns>();
        stage<Q, R, Ns, SIGN>(a, b, tw);
        stages<Q, Ns * R, SIGN>(b, a, tw);
    }
}

template <int Q, int Ns>
constexpr int stage_count()
{
    if constexpr (Ns < Q)
        return 1 + stage_count<Q, Ns * radix_of<Q / Ns>()>();
    else
        return 0;
}

// v <- sum_m v[m] exp(SIGN 2 pi i k m / Q)  (unnormalised)
template <int Q, int SIGN>
__device__ __forceinline__ void fft(float2 (&v)[Q], const float2 *__restrict__ tw)
{
    float2 t[Q];
    stages<Q, 1, SIGN>(v, t, tw);
    if constexpr (stage_count<Q, 1>() % 2 == 1) {
#pragma unroll
        for (int m = 0; m < Q; ++m)
            v[m] = t[m];
    }
}

}  // namespace tfft

enum { SRC_PLANES = 0, SRC_PSF = 1 };

// Half spectra of real tiles are Hermitian: on the columns kv = 0 and (Q even)
// kv = Q/2, row ku and row Q - ku hold complex conjugates.  The products of two
// such spectra keep the symmetry, so the contractions compute only the unique
// frequencies (rows ku <= Q/2 in full, the other rows without those columns)
// and the inverse transform reads the rest from their partners, conjugated.
// For Q = 28 that is 394 of 420 frequencies.
struct FreqMap {
    int QH;     // Q / 2 + 1 columns
    int L;      // full rows: ku <= Q / 2
    int m;      // columns of the other rows: 1 .. m
};

__host__ __device__ inline FreqMap freq_map(int Q)
{
    FreqMap f;
    f.QH = Q / 2 + 1;
    f.L = Q / 2 + 1;
    f.m = f.QH - ((Q % 2 == 0) ? 2 : 1);
    return f;
}

__host__ __device__ inline int unique_freqs(int Q)
{
    const FreqMap f = freq_map(Q);
    return f.L * f.QH + (Q - f.L) * f.m;
}

// Frequency index k = ku * QH + kv of the u-th unique frequency.
__device__ __forceinline__ int unique_freq(int u, const FreqMap &f)
{
    const int full = f.L * f.QH;
    if (u < full)
        return u;
    const int r = u - full;
    return (f.L + r / f.m) * f.QH + 1 + r % f.m;
}

// Whether frequency (ku, kv) is the conjugate of a unique one (its partner
// is row Q - ku of the same column).
template <int Q>
__device__ __forceinline__ bool freq_redundant(int ku, int kv)
{
    return ku > Q / 2 && (kv == 0 || (Q % 2 == 0 && kv == Q / 2));
}

// Loads in these kernels are issued in batches (the constants below) per thread
// before any of them is consumed, so a thread keeps that many requests in flight
// instead of waiting out the memory latency once per element.  Addresses are
// clamped to valid elements and unwanted values cleared with a bit mask (not a
// select, which the compiler would turn into a branch around the load).
// (deeper batches were measured slower: fewer blocks fit per CU)
// The forward transform loads its rows straight into registers instead.
static constexpr int kEpiBatch = 4;      // inverse: epilogue pixels per thread

// Frames whose tiles one launch covers.  Tiles of all frames are numbered
// consecutively (frame f owns tiles [tile0, tile0 + its tile count)); the
// contraction between the transforms treats them as one tile dimension, so the
// spectra stream once for the whole batch.
static constexpr int kMaxBatchJobs = 16;

// Per-pixel epilogues of the inverse transform (val = the transformed value,
// b = the frame's background):
//   EPI_STORE   dst = val + b
//   EPI_RATIO   dst = aux0 / (val + b), 0 where val + b <= 0   (aux0 = y)
//   EPI_UPDATE  dst = aux0 * val / aux1, 0 where aux1 <= 0     (x_old, A^T 1)
//   EPI_ISRA    dst = aux0 * aux1 / val, 0 where val <= 0      (x_old, A^T y)
enum { EPI_STORE = 0, EPI_RATIO = 1, EPI_UPDATE = 2, EPI_ISRA = 3 };

struct TileJob {
    const float *src;   // forward transform: source planes [planes][H][W]
    float *dst;         // inverse transform: destination (planes or image)
    const float *aux0;  // inverse transform: y (ratio) or x_old (updates)
    const float *aux1;  // inverse transform: A^T 1 (RL update) or A^T y (ISRA)
    float bg;           // inverse transform: background b
    int mode;           // inverse transform: epilogue
    int H, W, tiles_x, tile0;
    const int *skip;    // device flag (may be null): nonzero = skip this frame's tiles
};

struct TileBatch {
    int njobs;
    TileJob job[kMaxBatchJobs];
};

__device__ __forceinline__ int batch_job(const TileBatch &b, int tile)
{
    int f = 0;
    while (f + 1 < b.njobs && tile >= b.job[f + 1].tile0)
        ++f;
    return f;
}

__device__ __forceinline__ float keep_if(float v, bool keep)
{
    return __uint_as_float(__float_as_uint(v) & (keep ? 0xffffffffu : 0u));
}

// Per-(frequency, tile) maxima of tile spectra (split precision): every
// forward tile-DFT block stores the maxima of its columns at each frequency,
// rowpart[(grp * nt + tile) * Q*QH + k] (plain stores of the float bits,
// grp = the block's column group), and k_rowmax_reduce folds the groups into
// rowmax[k * nt + tile].  (Device-scope atomic maxima instead cost one 32-byte
// memory write each: 3.1 M per volume transform at 600 x 600 x 31.)
// Block (64 frequencies, tile) of 64 x 16 threads: thread (k, l) takes groups
// l, l + 16, ... (8 loads in flight), the 16 partial maxima then meet in LDS.
__global__ __launch_bounds__(1024) void k_rowmax_reduce(const unsigned *__restrict__ rowpart,
                                                        int ngrp, int nt, int nk,
                                                        const int *__restrict__ skip,
                                                        unsigned *__restrict__ rowmax)
{
    if (skip && *skip)
        return;
    __shared__ unsigned red[16][64];
    const int kl = threadIdx.x & 63, l = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + kl, tile = blockIdx.y;
    const int kc = min(k, nk - 1);
    unsigned m = 0u;
    for (int g0 = l; g0 < ngrp; g0 += 8 * 16) {
        unsigned v[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int g = min(g0 + 16 * b, ngrp - 1);  // a repeated group leaves the max
            v[b] = rowpart[((size_t)g * nt + tile) * nk + kc];
        }
#pragma unroll
        for (int b = 0; b < 8; ++b)
            m = max(m, v[b]);
    }
    red[l][kl] = m;
    __syncthreads();
    if (l == 0 && k < nk) {
#pragma unroll
        for (int q = 1; q < 16; ++q)
            m = max(m, red[q][kl]);
        rowmax[(size_t)k * nt + tile] = m;
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Remap the linear block id so that every XCD works through one contiguous
// range of work items: items that share cache lines then share an L2.
__device__ __forceinline__ int xcd_item(int bid, int n)
{
    constexpr int kXcds = 8;
    const int xcd = bid % kXcds, local = bid / kXcds;
    const int base = n / kXcds, rem = n % kXcds;
    return xcd * base + min(xcd, rem) + local;
}

// Forward real tile DFT of N interleaved phases, written as a half spectrum:
// out[obase + k * kstride + p], k = ku * (Q/2 + 1) + kv.
//   SRC_PLANES: one overlap-save tile of lenslet rows (plane j, row phase ar)
//               of a frame's [planes][H][W] array (frames and tiles from
//               `batch`; `src` unused), each row-pass thread loading its two
//               rows straight from memory; 1-D grid of nt * planes * N blocks,
//               work item = tile * (planes * N) + j*N + ar (the row phases of
//               one tile write adjacent pieces of every spectrum row and run
//               together on one XCD, so their partial cache lines merge in L2;
//               measured faster than keeping overlapping tiles together).
//               obase = (tile * KKo + j*N*N + ar*N), kstride = nt * KKo.
//   SRC_PSF:    the polyphase kernels G_{j,a->c}[D] = h[j][a][N*D + c - a + c0]
//               for output row phase cr and all column phases, placed
//               circularly in the tile; blockIdx = (cr, a, j); `src` is the
//               PSF; KKo is the row stride NNp of the spectra.
//               obase = ((j*N*N + a) * NNp + cr*N), kstride = KK * NNp.
//   rowpart (SRC_PLANES, may be null): the largest |re| or |im| the block
//   writes at frequency k (float bits) is stored at
//   rowpart[(grp * nt + tile) * Q*QH + k], grp = j*N + ar (see k_rowmax_reduce).
template <int Q>
__global__ __launch_bounds__(512) void k_r2c_fft(int mode, const TileBatch batch,
                                                  const float *__restrict__ src, int N, int T,
                                                  int hD, int nt, int KKo, int K, int c0, int KK,
                                                  float2 *__restrict__ out,
                                                  const float2 *__restrict__ twg,
                                                  unsigned *__restrict__ rowpart)
{
    constexpr int QH = Q / 2 + 1;
    extern __shared__ float smem[];
    float2 *tw = reinterpret_cast<float2 *>(smem);
    float *buf = smem + 2 * Q;
    float2 *Z = reinterpret_cast<float2 *>(buf);
    // SRC_PLANES loads its rows straight from memory: buf holds only Z (and,
    // at the end, the column magnitudes for rowmax)
    const int tid = threadIdx.x;
    for (int i = tid; i < Q; i += blockDim.x)
        tw[i] = twg[i];
    const int rowlen = Q * N;
    size_t obase, kstride;
    const float *plane = nullptr;
    int H = 0, W = 0, ly0 = 0, lx0 = 0, arow = 0, tile = 0, jar = 0;
    if (mode == SRC_PLANES) {
        const int item = xcd_item(blockIdx.x, gridDim.x);
        const int njar = gridDim.x / nt;
        tile = item / njar;
        jar = item % njar;
        const int j = jar / N;
        arow = jar % N;
        const TileJob &fj = batch.job[batch_job(batch, tile)];
        if (fj.skip && *fj.skip)
            return;   // block-uniform, before any barrier
        H = fj.H;
        W = fj.W;
        const int lt = tile - fj.tile0;
        ly0 = (lt / fj.tiles_x) * T - hD;
        lx0 = (lt % fj.tiles_x) * T - hD;
        plane = fj.src + (size_t)j * H * W;
        obase = (size_t)tile * KKo + (size_t)j * N * N + (size_t)arow * N;
        kstride = (size_t)nt * KKo;
    } else {
        const int cr = blockIdx.x, a = blockIdx.y, j = blockIdx.z;
        const int ar = a / N, ac = a % N;
        const float *hk = src + (((size_t)j * N + ar) * N + ac) * (size_t)K * K;
        for (int idx = tid; idx < Q * rowlen; idx += blockDim.x) {
            const int i = idx / rowlen, col = idx % rowlen;
            const int l = col / N, cc = col % N;
            const int Dr = (i <= hD) ? i : ((i >= Q - hD) ? i - Q : INT32_MIN);
            const int Dc = (l <= hD) ? l : ((l >= Q - hD) ? l - Q : INT32_MIN);
            float v = 0.f;
            if (Dr != INT32_MIN && Dc != INT32_MIN) {
                const int u = N * Dr + cr - ar + c0;
                const int vv = N * Dc + cc - ac + c0;
                if (u >= 0 && u < K && vv >= 0 && vv < K)
                    v = hk[(size_t)u * K + vv];
            }
            buf[idx] = v;
        }
        obase = ((size_t)j * N * N + a) * (size_t)KKo + (size_t)cr * N;
        kstride = (size_t)KK * KKo;
    }
    __syncthreads();
    // row pass: two real rows per thread packed as one complex sequence, rows
    // s and s + npairs (so that the lanes of a wave load consecutive rows s:
    // runs of N adjacent pixels per tile row)
    const int nseq = Q * N;
    const int npairs = (nseq + 1) / 2;
    float2 v[Q];
    int s0 = -1, s1 = -1;
    if (tid < npairs) {
        s0 = tid;
        s1 = (tid + npairs < nseq) ? tid + npairs : -1;
        const int i0 = s0 / N, p0 = s0 % N;
        const int i1 = s1 >= 0 ? s1 / N : 0, p1 = s1 >= 0 ? s1 % N : 0;
        if (mode == SRC_PLANES) {
            // the two rows straight from the plane: 2Q independent loads,
            // clamped addresses, values outside the image cleared by a mask
            const int pr0 = N * (ly0 + i0) + arow, pr1 = N * (ly0 + i1) + arow;
            const bool r0 = pr0 >= 0 && pr0 < H, r1 = s1 >= 0 && pr1 >= 0 && pr1 < H;
            const float *row0 = plane + (size_t)min(max(pr0, 0), H - 1) * W;
            const float *row1 = plane + (size_t)min(max(pr1, 0), H - 1) * W;
#pragma unroll
            for (int l = 0; l < Q; ++l) {
                const int pc0 = N * (lx0 + l) + p0, pc1 = N * (lx0 + l) + p1;
                const float a = row0[min(max(pc0, 0), W - 1)];
                const float b = row1[min(max(pc1, 0), W - 1)];
                v[l] = make_float2(keep_if(a, r0 && pc0 >= 0 && pc0 < W),
                                   keep_if(b, r1 && pc1 >= 0 && pc1 < W));
            }
        } else {
#pragma unroll
            for (int l = 0; l < Q; ++l) {
                const float a = buf[(size_t)i0 * rowlen + l * N + p0];
                const float b = s1 >= 0 ? buf[(size_t)i1 * rowlen + l * N + p1] : 0.f;
                v[l] = make_float2(a, b);
            }
        }
    }
    __syncthreads();  // every row is in registers: Z may now overwrite buf
    if (tid < npairs) {
        tfft::fft<Q, -1>(v, tw);
        const int i0 = s0 / N, p0 = s0 % N;
#pragma unroll
        for (int k = 0; k < QH; ++k) {
            const float2 zk = v[k], zm = v[(Q - k) % Q];
            // A = (Z[k] + conj(Z[-k])) / 2,  B = (Z[k] - conj(Z[-k])) / (2i)
            Z[((size_t)i0 * QH + k) * N + p0] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            if (s1 >= 0) {
                const int i1 = s1 / N, p1 = s1 % N;
                Z[((size_t)i1 * QH + k) * N + p1] =
                    make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
            }
        }
    }
    __syncthreads();
    // column pass: one complex column (kv, p) per thread
    if (tid < QH * N) {
        const int kv = tid / N, p = tid % N;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            v[i] = Z[((size_t)i * QH + kv) * N + p];
        tfft::fft<Q, -1>(v, tw);
#pragma unroll
        for (int ku = 0; ku < Q; ++ku)
            if (mode != SRC_PLANES || !freq_redundant<Q>(ku, kv))
                out[obase + (size_t)(ku * QH + kv) * kstride + p] = v[ku];
    }
    if (rowpart) {
        // the column magnitudes through LDS (Z has been read by every
        // thread), then the maximum over the N phases of each frequency
        __syncthreads();
        unsigned *mz = reinterpret_cast<unsigned *>(Z);  // [Q * QH][N]
        if (tid < QH * N) {
#pragma unroll
            for (int ku = 0; ku < Q; ++ku)
                mz[(size_t)ku * QH * N + tid] = __float_as_uint(fmaxf(fabsf(v[ku].x), fabsf(v[ku].y)));
        }
        __syncthreads();
        unsigned *dst = rowpart + ((size_t)jar * nt + tile) * (Q * QH);
        for (int i = tid; i < Q * QH; i += blockDim.x) {
            unsigned m = 0u;
            for (int q = 0; q < N; ++q)
                m = max(m, mz[(size_t)i * N + q]);
            dst[i] = m;
        }
    }
}

// Inverse tile DFT of N interleaved phases with the crop to the T x T valid
// lenslets and the per-pixel epilogue (see k_c2r for the modes).  The spectrum
// of column q = j*N*N + ar*N + p at frequency k is
// sum_s spec[s * split_stride + k * sk + tile * stile + q * sc].
// 1-D grid of nt * planes * N blocks, work item = tile * (planes * N) + j*N + ar
// (consecutive phases of one tile read adjacent spectra and share an XCD).
template <int Q>
__global__ __launch_bounds__(512) void k_c2r_fft(const TileBatch batch,
                                                  const float2 *__restrict__ spec,
                                                  size_t split_stride, int nsplit, size_t sk,
                                                  size_t stile, size_t sc, int N, int planes,
                                                  int T, int hD, const float2 *__restrict__ twg,
                                                  int stage)
{
    constexpr int QH = Q / 2 + 1;
    extern __shared__ float smem[];
    float2 *tw = reinterpret_cast<float2 *>(smem);
    float2 *Zs = tw + Q;                                    // [T][QH][N]
    float *obuf = reinterpret_cast<float *>(Zs + (size_t)T * QH * N);  // [T][T][N]
    const int tid = threadIdx.x;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    const int tile = item / (planes * N), jar = item % (planes * N);
    const int j = jar / N, ar = jar % N;
    const TileJob &fj = batch.job[batch_job(batch, tile)];
    if (fj.skip && *fj.skip)
        return;   // block-uniform, before any barrier
    const int H = fj.H, W = fj.W, lt = tile - fj.tile0;
    const int ty = lt / fj.tiles_x, tx = lt % fj.tiles_x;
    float *__restrict__ dst = fj.dst;
    const float *__restrict__ aux0 = fj.aux0;
    const float *__restrict__ aux1 = fj.aux1;
    const int mode = fj.mode;
    const float bg = fj.bg;
    // epilogue geometry: whole pixel rows of the tile; the plane's base
    // pointers are uniform and pixel offsets are 32-bit (a plane is < 2^30 pixels)
    const int Ly = H / N, Lx = W / N;
    const int rowpix = T * N;
    const int ototal = T * rowpix;
    const size_t plane_off = (mode == EPI_RATIO) ? 0 : (size_t)j * H * W;
    const float *__restrict__ a0p = aux0 + plane_off;
    const float *__restrict__ a1p = aux1 + plane_off;
    float *__restrict__ dp = dst + plane_off;
    // pixel offset of output idx (clamped into the image) and whether it is kept
    auto epi_pixel = [&](int idx, bool &ok) -> unsigned {
        const int ti = idx / rowpix, rem = idx % rowpix;
        const int Lr = ty * T + ti, Lc = tx * T + rem / N;
        ok = Lr < Ly && Lc < Lx;
        const int pr = min(N * Lr + ar, H - 1), pc = min(N * tx * T + rem, W - 1);
        return (unsigned)pr * (unsigned)W + (unsigned)pc;
    };
    // With `stage`, the epilogue inputs go straight from memory into LDS
    // (a0s, a1s after obuf, 64 pixels per wave-wide load), issued right after
    // the spectrum loads so that their latency overlaps both transforms; they
    // are waited for before the barrier that precedes the epilogue.
    const int ostage = (ototal + 63) / 64 * 64;
    float *a0s = obuf + (size_t)T * T * N, *a1s = a0s + ostage;
    for (int i = tid; i < Q; i += blockDim.x)
        tw[i] = twg[i];
    __syncthreads();
    const size_t kkbase = (size_t)j * N * N + (size_t)ar * N;
    float2 v[Q];
    // inverse along tile rows (ku -> i) for column (kv, p), keeping the T valid
    // rows: each thread loads its Q spectrum values straight from memory (Q
    // independent loads in flight, no staging buffer), summing split partials
    const bool colthr = tid < QH * N;
    const int kv = tid / N, p = tid % N;
    if (colthr) {
        // a uniform base per row ku (scalar registers) plus one 32-bit byte
        // offset per thread (the launch keeps QH * sk * 8 below 2^32): the
        // loads need no 64-bit address per element
        const char *blk = reinterpret_cast<const char *>(spec + tile * stile + kkbase * sc);
        const unsigned toff = (unsigned)(((size_t)kv * sk + (size_t)p * sc) * sizeof(float2));
        const size_t kstep = (size_t)QH * sk * sizeof(float2);
#pragma unroll
        for (int ku = 0; ku < Q; ++ku)
            v[ku] = *reinterpret_cast<const float2 *>(blk + ku * kstep + toff);
        for (int s = 1; s < nsplit; ++s) {
            const char *blks = blk + (size_t)s * split_stride * sizeof(float2);
            // partials in chunks of 8 loads (a second Q-long array would spill)
#pragma unroll
            for (int k0 = 0; k0 < Q; k0 += 8) {
                float2 part[8];
#pragma unroll
                for (int d = 0; d < 8; ++d)
                    if (k0 + d < Q)
                        part[d] = *reinterpret_cast<const float2 *>(blks + (k0 + d) * kstep + toff);
#pragma unroll
                for (int d = 0; d < 8; ++d)
                    if (k0 + d < Q) {
                        v[k0 + d].x += part[d].x;
                        v[k0 + d].y += part[d].y;
                    }
            }
        }
    }
    // (every lane of a wave takes part in a direct-to-LDS load)
    if (stage && mode != EPI_STORE) {
        const int nw = blockDim.x >> 6, wave = tid >> 6, lane = tid & 63;
        for (int c = wave; c < ostage / 64; c += nw) {
            bool ok;
            const unsigned o = epi_pixel(min(64 * c + lane, ototal - 1), ok);
            __builtin_amdgcn_global_load_lds(
                a0p + o, (__attribute__((address_space(3))) void *)(a0s + 64 * c), 4, 0, 0);
            if (mode >= EPI_UPDATE)
                __builtin_amdgcn_global_load_lds(
                    a1p + o, (__attribute__((address_space(3))) void *)(a1s + 64 * c), 4, 0, 0);
        }
    }
    if (colthr) {
        // the redundant rows of the columns kv = 0 and kv = Q/2 were never
        // written (see FreqMap): the conjugates of their partner rows, which
        // this thread holds, replace whatever was read there (a select, so
        // stale values cannot leak)
        const bool edge = kv == 0 || (Q % 2 == 0 && kv == Q / 2);
#pragma unroll
        for (int ku = Q / 2 + 1; ku < Q; ++ku) {
            const float2 c = v[Q - ku];
            v[ku].x = edge ? c.x : v[ku].x;
            v[ku].y = edge ? -c.y : v[ku].y;
        }
        tfft::fft<Q, 1>(v, tw);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int ti = i - hD;
            if (ti >= 0 && ti < T)
                Zs[((size_t)ti * QH + kv) * N + p] = v[i];
        }
    }
    __syncthreads();
    // inverse real transform along tile columns: two Hermitian rows per thread
    const int nrow = T * N;
    const int npairs = (nrow + 1) / 2;
    const float scale = 1.0f / (float)(Q * Q);
    if (tid < npairs) {
        const int r0 = 2 * tid, r1 = (2 * tid + 1 < nrow) ? 2 * tid + 1 : -1;
        const int ti0 = r0 / N, p0 = r0 % N;
        const int ti1 = r1 >= 0 ? r1 / N : 0, p1 = r1 >= 0 ? r1 % N : 0;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const bool lo = k < QH;
            const int kk = lo ? k : Q - k;
            float2 a = Zs[((size_t)ti0 * QH + kk) * N + p0];
            float2 b = r1 >= 0 ? Zs[((size_t)ti1 * QH + kk) * N + p1] : make_float2(0.f, 0.f);
            if (k == 0 || 2 * k == Q) {
                a.y = 0.f;
                b.y = 0.f;
            }
            if (!lo) {
                a.y = -a.y;
                b.y = -b.y;
            }
            // a + i b
            v[k] = make_float2(a.x - b.y, a.y + b.x);
        }
        tfft::fft<Q, 1>(v, tw);
#pragma unroll
        for (int l = 0; l < Q; ++l) {
            const int tl = l - hD;
            if (tl >= 0 && tl < T) {
                obuf[((size_t)ti0 * T + tl) * N + p0] = v[l].x * scale;
                if (r1 >= 0)
                    obuf[((size_t)ti1 * T + tl) * N + p1] = v[l].y * scale;
            }
        }
    }
    if (stage)  // this wave's direct-to-LDS loads have landed (vmcnt 0)
        __builtin_amdgcn_s_waitcnt(0x0f70);
    __syncthreads();
    if (stage) {
        for (int idx = tid; idx < ototal; idx += blockDim.x) {
            bool ok;
            const unsigned o = epi_pixel(idx, ok);
            if (!ok)
                continue;
            const float val = obuf[idx];
            if (mode == EPI_STORE) {
                dp[o] = val + bg;
            } else if (mode == EPI_RATIO) {
                const float m = val + bg;
                dp[o] = m > 0.f ? a0s[idx] / m : 0.f;
            } else if (mode == EPI_UPDATE) {
                const float c = a1s[idx];
                dp[o] = c > 0.f ? a0s[idx] * val / c : 0.f;
            } else {
                dp[o] = val > 0.f ? a0s[idx] * a1s[idx] / val : 0.f;
            }
        }
        return;
    }
    // coalesced epilogue, inputs loaded in batches
    for (int base = tid; base < ototal; base += kEpiBatch * blockDim.x) {
        unsigned o[kEpiBatch];
        bool ok[kEpiBatch];
        float a0[kEpiBatch], a1[kEpiBatch];
#pragma unroll
        for (int b = 0; b < kEpiBatch; ++b) {
            const int idx = min(base + b * (int)blockDim.x, ototal - 1);
            o[b] = epi_pixel(idx, ok[b]);
            ok[b] = ok[b] && base + b * (int)blockDim.x < ototal;
            a0[b] = (mode != EPI_STORE) ? a0p[o[b]] : 0.f;
            a1[b] = (mode >= EPI_UPDATE) ? a1p[o[b]] : 0.f;
        }
#pragma unroll
        for (int b = 0; b < kEpiBatch; ++b) {
            if (!ok[b])
                continue;
            const float val = obuf[base + b * (int)blockDim.x];
            if (mode == EPI_STORE) {
                dp[o[b]] = val + bg;
            } else if (mode == EPI_RATIO) {
                const float m = val + bg;
                dp[o[b]] = m > 0.f ? a0[b] / m : 0.f;
            } else if (mode == EPI_UPDATE) {
                dp[o[b]] = a1[b] > 0.f ? a0[b] * val / a1[b] : 0.f;
            } else {
                dp[o[b]] = val > 0.f ? a0[b] * a1[b] / val : 0.f;
            }
        }
    }
}
