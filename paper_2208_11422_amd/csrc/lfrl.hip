// lfrl.hip - light-field Richardson-Lucy deconvolution on MI355X (gfx950).
//
// The forward light-field projection (every depth plane and every lenslet-
// relative phase convolved with its own PSF, summed into one image) is computed
// on the lenslet grid.  Write a pixel index as p = N*L + c (lenslet L, phase c)
// per axis.  Then
//     y_c[L] = sum_{j,a} (G_{j,a->c} * x_{j,a})[L],
//     G_{j,a->c}[D] = h[j][a][N*D + c - a + c0],
// a sum of small 2-D convolutions on the lenslet grid with polyphase kernels
// of R x R taps, R = 2*floor((c0 + N - 1)/N) + 1.  With overlap-save tiles of Q
// lenslets and half-spectrum DFTs, every frequency k of a tile is a dense
// complex contraction
//     Y_k[c][tile] = sum_{(j,a)} G_k[(j,a)][c] X_k[(j,a)][tile]          (forward)
//     B_k[(j,a)][tile] = sum_c conj(G_k[(j,a)][c]) R_k[c][tile]          (adjoint)
// The spectra G_k are built once per PSF set (the PSF stays on the card and is
// reused by every reconstruction, Fig. 1) and kept in two layouts, one per
// direction, so each contraction streams them with unit-stride loads.
//
// Pipeline of one Richardson-Lucy iteration (sec. 1 / sec. 2.1, all on device):
//   k_vol_r2c(x) -> k_contract_fwd -> k_c2r[ratio: rho = y / (A x)]
//   k_vol_r2c(rho) -> k_contract_adj -> k_c2r[update: x *= A^T rho / A^T 1]
//   metric (sec. 2.2): k_mip -> k_dct_rows -> k_metric_coeffs
//                      -> k_metric_final (entropy + stop rule) -> k_cond_copy
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lfrl.h"
#include "tile_fft.hpp"

#ifndef LFRL_KARA
#define LFRL_KARA 1
#endif

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return set_error(LFRL_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH_CHECK(name)                                                             \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess)                                                          \
            return set_error(LFRL_ERR_DEVICE, "launch of %s failed: %s", name, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// limits
// ---------------------------------------------------------------------------
static constexpr int kMaxQ = 64;        // DFT tile side
static constexpr int kMaxNN = 256;      // nnum^2 (one thread per output phase)
static constexpr int kMaxTrace = 4096;  // iterations recorded per deconvolve call
static constexpr int kMetricChunks = 8;   // row chunks of the DCT row transform
static constexpr int kMaxMetricLegs = 256;
static constexpr int kMetricBigCoefs = 16384;  // above: entropy summed over many blocks
static constexpr float kWeakThreshold = 1e-2f;  // weak voxel: A^T 1 < this * max A^T 1

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
struct Geo {
    int N, Nz, K, c0, hD, R, Q, QH, T, nf, NN, NNp, KK, KKs, NCp, KKb;
    int NCm;  // adjoint reduction on the matrix cores (a multiple of 8)
    int xc;   // the lone reduction index past them (summed on the vector ALU), or -1
    int NNm;  // forward output columns on the matrix cores (a multiple of 16)
    int xcol; // the lone output column past them (summed on the vector ALU), or -1
};

static void geo_init(Geo &g, int N, int Nz, int K, int Q)
{
    g.N = N;
    g.Nz = Nz;
    g.K = K;
    g.c0 = (K - 1) / 2;
    g.hD = (g.c0 + N - 1) / N;
    g.R = 2 * g.hD + 1;
    g.Q = Q;
    g.QH = Q / 2 + 1;
    g.T = Q - g.R + 1;
    g.nf = Q * g.QH;
    g.NN = N * N;
    g.NNp = (g.NN + 15) / 16 * 16;  // forward spectra row stride (aligned 16-column blocks)
    g.KK = g.NN * Nz;
    g.KKs = (g.KK + 31) / 32 * 32;  // row stride of the volume tile spectra
    g.NCp = (g.NN + 7) / 8 * 8;     // adjoint reduction length in fragment pairs
    // a single index past the last full group of 8 (NN = 225 for Nnum 15) is not
    // worth 7 zero-padded fragment rows: it is added on the vector ALU instead
    g.NCm = (g.NN % 8 == 1 && g.NN > 8) ? g.NN - 1 : g.NCp;
    g.xc = g.NCm < g.NN ? g.NN - 1 : -1;
    // likewise a single forward output column past the last full block of 16
    g.NNm = (g.NN % 16 == 1 && g.NN > 16) ? g.NN - 1 : g.NNp;
    g.xcol = g.NNm < g.NN ? g.NN - 1 : -1;
    g.KKb = (g.KK + 15) / 16 * 16;  // adjoint output columns in 16-column blocks
}

struct Tiles {
    int Ly, Lx, ty, tx, nt;
};

static Tiles tiles_for(const Geo &g, int h, int w)
{
    Tiles t;
    t.Ly = h / g.N;
    t.Lx = w / g.N;
    t.ty = (t.Ly + g.T - 1) / g.T;
    t.tx = (t.Lx + g.T - 1) / g.T;
    t.nt = t.ty * t.tx;
    return t;
}

// LDS bytes of the r2c / c2r tile kernels.
static size_t lds_r2c(const Geo &g)
{
    size_t in = (size_t)g.Q * g.Q * g.N;
    in = (in + 1) & ~(size_t)1;
    return in * 4 + (size_t)g.Q * g.QH * g.N * 8 + (size_t)g.Q * 8;
}

static size_t lds_c2r(const Geo &g)
{
    return (size_t)g.Q * g.QH * g.N * 8 + (size_t)g.T * g.QH * g.N * 8 + (size_t)g.Q * 8;
}


// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Row pass of a real Q x Q tile DFT for NP interleaved phases held in LDS as
// raw pixel rows: in[i][l*NP + p].  Produces the half spectrum along the row:
// Z[i][kv][p] = sum_l in[i][l*NP + p] * exp(-2 pi i l kv / Q), kv <= Q/2.
__device__ __forceinline__ void dft_rows_r2c(const float *in, float2 *Z, const float2 *tw,
                                             int Q, int QH, int NP)
{
    const int total = Q * QH * NP;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int p = idx % NP;
        const int kv = (idx / NP) % QH;
        const int i = idx / (NP * QH);
        const float *row = in + (size_t)i * Q * NP + p;
        float re = 0.f, im = 0.f;
        int m = 0;
        for (int l = 0; l < Q; ++l) {
            const float v = row[l * NP];
            const float2 w = tw[m];
            re = fmaf(v, w.x, re);
            im = fmaf(-v, w.y, im);
            m += kv;
            if (m >= Q)
                m -= Q;
        }
        Z[idx] = make_float2(re, im);
    }
}

// ---------------------------------------------------------------------------
// plan-time kernels
// ---------------------------------------------------------------------------

// Polyphase kernels of one (plane j, source phase a) for one output row phase
// cr, all output column phases cc: the R x R taps G[D] = h[j][a][N*D + c - a + c0]
// placed circularly (D mod Q) in a Q x Q tile, transformed, and written as
// Gf[k][kk][c] with kk = j*N*N + a, c = cr*N + cc (rows of NNp >= N*N entries).
__global__ void k_psf_r2c(const float *__restrict__ psf, int N, int K, int c0, int hD, int Q,
                          int QH, int KK, int NNp, float2 *__restrict__ Gf,
                          const float2 *__restrict__ twg)
{
    extern __shared__ float smem[];
    const int cr = blockIdx.x;
    const int a = blockIdx.y;
    const int j = blockIdx.z;
    const int ar = a / N, ac = a % N;
    const int rowlen = Q * N;
    size_t in_n = (size_t)Q * rowlen;
    in_n = (in_n + 1) & ~(size_t)1;
    float *in = smem;
    float2 *Z = reinterpret_cast<float2 *>(smem + in_n);
    float2 *tw = Z + (size_t)Q * QH * N;
    for (int i = threadIdx.x; i < Q; i += blockDim.x)
        tw[i] = twg[i];
    const float *hk = psf + (((size_t)j * N + ar) * N + ac) * (size_t)K * K;
    for (int idx = threadIdx.x; idx < Q * rowlen; idx += blockDim.x) {
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
        in[idx] = v;
    }
    __syncthreads();
    dft_rows_r2c(in, Z, tw, Q, QH, N);
    __syncthreads();
    const size_t kk = (size_t)j * N * N + a;
    const int total = Q * QH * N;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int p = idx % N;
        const int kv = (idx / N) % QH;
        const int ku = idx / (N * QH);
        float re = 0.f, im = 0.f;
        int m = 0;
        for (int i = 0; i < Q; ++i) {
            const float2 z = Z[((size_t)i * QH + kv) * N + p];
            const float2 w = tw[m];
            re = fmaf(z.x, w.x, fmaf(z.y, w.y, re));
            im = fmaf(z.y, w.x, fmaf(-z.x, w.y, im));
            m += ku;
            if (m >= Q)
                m -= Q;
        }
        const size_t k = (size_t)ku * QH + kv;
        Gf[(k * KK + kk) * NNp + (size_t)cr * N + p] = make_float2(re, im);
    }
}

// Gb[k][c][kk] = Gf[k][kk][c]: per-frequency transpose through LDS (Gf rows
// hold NNp entries, Gb rows KK).
__global__ void k_transpose_spec(const float2 *__restrict__ Gf, float2 *__restrict__ Gb,
                                 int KK, int NN, int NNp)
{
    __shared__ float2 tile[32][33];
    const size_t k = blockIdx.z;
    const int c0 = blockIdx.x * 32, kk0 = blockIdx.y * 32;
    const float2 *src = Gf + k * (size_t)KK * NNp;
    float2 *dst = Gb + k * (size_t)KK * NN;
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int kk = kk0 + r, c = c0 + threadIdx.x;
        if (kk < KK && c < NN)
            tile[r][threadIdx.x] = src[(size_t)kk * NNp + c];
    }
    __syncthreads();
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int c = c0 + r, kk = kk0 + threadIdx.x;
        if (kk < KK && c < NN)
            dst[(size_t)c * KK + kk] = tile[threadIdx.x][r];
    }
}

// ---------------------------------------------------------------------------
// per-iteration kernels
// ---------------------------------------------------------------------------

// Gather one overlap-save tile of lenslet rows (plane j, row phase ar, all N
// column phases) from a [planes][H][W] array and write its half spectrum:
// out[k][tile][kk] with kk = j*N*N + ar*N + ac.  Lenslets outside the image
// are zero (linear, not circular, convolution).
__global__ void k_vol_r2c(const TileBatch batch, int N, int Q, int QH, int T, int hD, int nt,
                          int KKo, float2 *__restrict__ out, const float2 *__restrict__ twg)
{
    extern __shared__ float smem[];
    const int tile = blockIdx.x;
    const int j = blockIdx.y / N, ar = blockIdx.y % N;
    const TileJob &fj = batch.job[batch_job(batch, tile)];
    if (fj.skip && *fj.skip)
        return;   // block-uniform, before any barrier
    const int H = fj.H, W = fj.W, lt = tile - fj.tile0;
    const int ty = lt / fj.tiles_x, tx = lt % fj.tiles_x;
    const int ly0 = ty * T - hD, lx0 = tx * T - hD;
    const int rowlen = Q * N;
    size_t in_n = (size_t)Q * rowlen;
    in_n = (in_n + 1) & ~(size_t)1;
    float *in = smem;
    float2 *Z = reinterpret_cast<float2 *>(smem + in_n);
    float2 *tw = Z + (size_t)Q * QH * N;
    for (int i = threadIdx.x; i < Q; i += blockDim.x)
        tw[i] = twg[i];
    const float *plane = fj.src + (size_t)j * H * W;
    for (int idx = threadIdx.x; idx < Q * rowlen; idx += blockDim.x) {
        const int i = idx / rowlen, col = idx % rowlen;
        const int pr = N * (ly0 + i) + ar;
        const int pc = N * lx0 + col;
        float v = 0.f;
        if (pr >= 0 && pr < H && pc >= 0 && pc < W)
            v = plane[(size_t)pr * W + pc];
        in[idx] = v;
    }
    __syncthreads();
    dft_rows_r2c(in, Z, tw, Q, QH, N);
    __syncthreads();
    const size_t kkbase = (size_t)j * N * N + (size_t)ar * N;
    const int total = Q * QH * N;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int p = idx % N;
        const int kv = (idx / N) % QH;
        const int ku = idx / (N * QH);
        float re = 0.f, im = 0.f;
        int m = 0;
        for (int i = 0; i < Q; ++i) {
            const float2 z = Z[((size_t)i * QH + kv) * N + p];
            const float2 w = tw[m];
            re = fmaf(z.x, w.x, fmaf(z.y, w.y, re));
            im = fmaf(z.y, w.x, fmaf(-z.x, w.y, im));
            m += ku;
            if (m >= Q)
                m -= Q;
        }
        const size_t k = (size_t)ku * QH + kv;
        out[(k * nt + tile) * KKo + kkbase + p] = make_float2(re, im);
    }
}


// Inverse tile DFT and scatter of the valid T x T lenslets of one tile for
// plane j and row phase ar (all N column phases).  The spectrum of column
// index q = j*N*N + ar*N + p at frequency k is
// sum_s spec[s*split_stride + k*sk + tile*stile + q*sc] (split-K partials).
// Epilogues:  STORE  dst[j][pr][pc] = v
//             RATIO  dst[pr][pc] = v > 0 ? aux0[pr][pc] / v : 0   (rho = y / A x)
//             UPDATE dst[j][pr][pc] = aux1 > 0 ? aux0 * v / aux1 : 0
//                    (x_new = x_old * A^T rho / A^T 1)
__global__ void k_c2r(const TileBatch batch, const float2 *__restrict__ spec, size_t split_stride,
                      int nsplit, size_t sk, size_t stile, size_t sc, int N, int Q, int QH, int T,
                      int hD, const float2 *__restrict__ twg)
{
    extern __shared__ float smem[];
    const int tile = blockIdx.x;
    const int j = blockIdx.y / N, ar = blockIdx.y % N;
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
    float2 *X = reinterpret_cast<float2 *>(smem);
    float2 *Z = X + (size_t)Q * QH * N;
    float2 *tw = Z + (size_t)T * QH * N;
    for (int i = threadIdx.x; i < Q; i += blockDim.x)
        tw[i] = twg[i];
    const size_t kkbase = (size_t)j * N * N + (size_t)ar * N;
    const int total = Q * QH * N;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int p = idx % N;
        const int kq = idx / N;
        const int ku = kq / QH, kv = kq % QH;
        // redundant frequencies (see FreqMap) from their conjugate partners
        const bool red = ku > Q / 2 && (kv == 0 || (Q % 2 == 0 && kv == Q / 2));
        const size_t k = red ? (size_t)(Q - ku) * QH + kv : (size_t)kq;
        const size_t off = k * sk + tile * stile + (kkbase + p) * sc;
        float2 acc = spec[off];
        for (int s = 1; s < nsplit; ++s) {
            const float2 v = spec[off + s * split_stride];
            acc.x += v.x;
            acc.y += v.y;
        }
        if (red)
            acc.y = -acc.y;
        X[idx] = acc;
    }
    __syncthreads();
    // inverse DFT along the tile rows (ku -> i), only for the T valid rows
    const int ztotal = T * QH * N;
    for (int idx = threadIdx.x; idx < ztotal; idx += blockDim.x) {
        const int p = idx % N;
        const int kv = (idx / N) % QH;
        const int ti = idx / (N * QH);
        const int i = hD + ti;
        float re = 0.f, im = 0.f;
        int m = 0;
        for (int ku = 0; ku < Q; ++ku) {
            const float2 x = X[((size_t)ku * QH + kv) * N + p];
            const float2 w = tw[m];
            re = fmaf(x.x, w.x, fmaf(-x.y, w.y, re));
            im = fmaf(x.x, w.y, fmaf(x.y, w.x, im));
            m += i;
            if (m >= Q)
                m -= Q;
        }
        Z[idx] = make_float2(re, im);
    }
    __syncthreads();
    // inverse real DFT along the tile columns (Hermitian half spectrum)
    const float scale = 1.0f / (float)(Q * Q);
    const int Ly = H / N, Lx = W / N;
    const int otot = T * T * N;
    for (int idx = threadIdx.x; idx < otot; idx += blockDim.x) {
        const int p = idx % N;
        const int tl = (idx / N) % T;
        const int ti = idx / (N * T);
        const int l = hD + tl;
        const int Lr = ty * T + ti, Lc = tx * T + tl;
        if (Lr >= Ly || Lc >= Lx)
            continue;
        float v = 0.f;
        int m = 0;
        for (int kv = 0; kv < QH; ++kv) {
            const float2 z = Z[((size_t)ti * QH + kv) * N + p];
            const float2 w = tw[m];
            const float wt = (kv == 0 || 2 * kv == Q) ? 1.f : 2.f;
            v = fmaf(wt, fmaf(z.x, w.x, -z.y * w.y), v);
            m += l;
            if (m >= Q)
                m -= Q;
        }
        v *= scale;
        const int pr = N * Lr + ar, pc = N * Lc + p;
        const size_t pix = (size_t)pr * W + pc;
        if (mode == EPI_STORE) {
            dst[(size_t)j * H * W + pix] = v + bg;
        } else if (mode == EPI_RATIO) {
            const float m = v + bg;
            dst[pix] = m > 0.f ? aux0[pix] / m : 0.f;
        } else if (mode == EPI_UPDATE) {
            const size_t o = (size_t)j * H * W + pix;
            const float c = aux1[o];
            dst[o] = c > 0.f ? aux0[o] * v / c : 0.f;
        } else {
            const size_t o = (size_t)j * H * W + pix;
            dst[o] = v > 0.f ? aux0[o] * aux1[o] / v : 0.f;
        }
    }
}

// ---------------------------------------------------------------------------
// spectral contractions on FP32 matrix cores
// ---------------------------------------------------------------------------
// Each complex product is four real v_mfma_f32_16x16x4f32 products (full FP32
// inputs, FP32 accumulation).  Fragment layouts of that instruction (wave64):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[4 * (l / 16) + i][l % 16] in element i.
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Fragment loads of the adjoint contraction, non-temporal: they are read once
// per launch and far exceed the caches (measured faster; the same hint made
// the forward contraction and the adjoint's stores slower)
__device__ __forceinline__ float4 adj_load4(const float4 *p)
{
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}


__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Block coordinates of a contraction launch on a (nf, y, tile groups) grid:
// frequency k, the y index (K chunk or kk ranges) and the tile group.  With
// several tile groups (batched frames), the groups of one (k, y) are
// consecutive work items of one XCD: they stream the same PSF fragments at the
// same time, so HBM delivers each fragment about once and that XCD's L2 the
// other times, instead of once per group.  A single group keeps the plain
// order.
__device__ __forceinline__ void contraction_block(int &k, int &y, int &tg)
{
    const int ntg = gridDim.z;
    if (ntg == 1) {
        k = blockIdx.x;
        y = blockIdx.y;
        tg = 0;
        return;
    }
    const int n = gridDim.x * gridDim.y * ntg;
    const int lin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const int item = xcd_item(lin, n);
    tg = item % ntg;
    const int rest = item / ntg;
    k = rest % gridDim.x;
    y = rest / gridDim.x;
}

#include "contract_split.hpp"

// Spectra in fragment order.  One load instruction of a wave then reads one
// contiguous kilobyte: each lane takes 16 bytes, the two complex values it
// feeds to two consecutive MFMA steps.  (Row-major spectra with 8-byte loads
// touch four separate 128-byte pieces per instruction and stream at about
// 70% of the rate of contiguous 16-byte loads.)
//   forward  Ff[k][p][cb][lane] = {G(8p+2q, 16cb+col), G(8p+2q+1, 16cb+col)},
//            G(kk, c) = Gf[k][kk][c], p < KKs/8, cb < NNp/16;
//   adjoint  fragment (p, kb) of frequency k = {H(8p+2q, 16kb+col), H(8p+2q+1, 16kb+col)},
//            H(c, kk) = Gb[k][c][kk], p < NCp/8, kb < KKb/16, stored range-major
//            (adj_frag);
// with q = lane / 16, col = lane % 16 and zeros outside the valid ranges.
// The reduction index kk (forward) or c (adjoint) of MFMA step 2u + h is
// 8u + 2q + h for lane group q: the sums are the same, taken in this order.
__global__ void k_pack_fwd_f32(const float2 *__restrict__ Gf, int KK, int NNp, int ncb, int KKs,
                               float4 *__restrict__ Ff, size_t total)
{
    const int np = KKs / 8;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const int lane = (int)(i % 64);
        const size_t r = i / 64;
        const int cb = (int)(r % ncb);
        const size_t r2 = r / ncb;
        const int p = (int)(r2 % np);
        const size_t k = r2 / np;
        const int kk = 8 * p + 2 * (lane >> 4), c = 16 * cb + (lane & 15);
        const float2 *gk = Gf + k * (size_t)KK * NNp;
        const float2 a = kk < KK ? gk[(size_t)kk * NNp + c] : make_float2(0.f, 0.f);
        const float2 b = kk + 1 < KK ? gk[(size_t)(kk + 1) * NNp + c] : make_float2(0.f, 0.f);
        Ff[i] = make_float4(a.x, a.y, b.x, b.y);
    }
}

// Column xcol of the forward spectra, Gx[k][kk] = Gf[k][kk][xcol] (0 past KK):
// the lone output column the forward contraction sums on the vector ALU.
__global__ void k_spec_column(const float2 *__restrict__ Gf, int KK, int NNp, int KKs, int xcol,
                              float2 *__restrict__ Gx, size_t total)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t k = i / KKs;
        const int kk = (int)(i % KKs);
        Gx[i] = kk < KK ? Gf[(k * KK + kk) * NNp + xcol] : make_float2(0.f, 0.f);
    }
}

// Adjoint fragments, range-major so that the fragments one block of the
// adjoint contraction reads (RB column blocks of every pair) are contiguous:
// range rb = kb / RB starts at fragment rb * RB * np; inside it fragment
// (p, j = kb % RB) sits at p * w + j, w = min(RB, nkb - rb * RB).
__device__ __forceinline__ size_t adj_frag(int p, int kb, int np, int nkb, int RB)
{
    const int rb = kb / RB, j = kb - rb * RB;
    const int w = min(RB, nkb - rb * RB);
    return (size_t)rb * RB * np + (size_t)p * w + j;
}

__global__ void k_pack_adj_f32(const float2 *__restrict__ Gb, int NN, int KK, int NCp, int KKb,
                               int RB, float4 *__restrict__ Fb, size_t total)
{
    const int nkb = KKb / 16, np = NCp / 8;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const int lane = (int)(i % 64);
        const size_t r = i / 64;
        const int kb = (int)(r % nkb);
        const size_t r2 = r / nkb;
        const int p = (int)(r2 % np);
        const size_t k = r2 / np;
        const int c = 8 * p + 2 * (lane >> 4), kk = 16 * kb + (lane & 15);
        const float2 *gk = Gb + k * (size_t)NN * KK;
        const bool okk = kk < KK;
        const float2 a = okk && c < NN ? gk[(size_t)c * KK + kk] : make_float2(0.f, 0.f);
        const float2 b = okk && c + 1 < NN ? gk[(size_t)(c + 1) * KK + kk] : make_float2(0.f, 0.f);
        Fb[(k * np * nkb + adj_frag(p, kb, np, nkb, RB)) * 64 + lane] = make_float4(a.x, a.y, b.x, b.y);
    }
}

__device__ __forceinline__ float mask_f(float v, bool keep)
{
    return __uint_as_float(__float_as_uint(v) & (keep ? 0xffffffffu : 0u));
}

// Forward contraction for one frequency k and one reduction chunk s, computed
// transposed so that tiles are the MFMA rows:
//   Yp[s][k][t][c] = sum_{kk in chunk} X[k][t][kk] * Gf[k][kk][c]
// A = X: every wave needs the same 16 x 8U fragment per register group, so
// the block loads it once, coalesced (16-byte loads along the tile rows), and
// keeps it in LDS in fragment order (double-buffered, one barrier per group).
// The block must have at least 64 * U threads (U waves): one value each.
// B = Ff fragments, CB blocks of 16 columns per wave, loaded straight into
// registers and double-buffered.  X past KK (padding that may hold stale
// data) is cleared by a bit mask when it is written to LDS.  Outputs for
// t >= nt or c >= NN are not stored.
template <int CB, int U>
__global__ __launch_bounds__(512) void k_contract_fwd(const float4 *__restrict__ Ff,
                                                      const float2 *__restrict__ X,
                                                      float2 *__restrict__ Yp, int NN, int NNp,
                                                      int KK, int KKs, int nt, int nf, int kchunk,
                                                      const int *__restrict__ skip, FreqMap fm,
                                                      const float4 *__restrict__ Gx4, int xcol)
{
    if (skip && *skip)
        return;
    __shared__ float4 la[2][U][64];
    int k, s, tg;
    contraction_block(k, s, tg);
    k = unique_freq(k, fm);
    const int t0 = tg * 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int ncb = NNp / 16;
    const int p0 = s * (kchunk / 8);
    const int p1 = min((KK + 7) / 8, p0 + kchunk / 8);
    const int npairs = p1 - p0;
    const int ngroups = (npairs + U - 1) / U;
    if (npairs <= 0)
        return;
    // staging: thread i handles float4 j = i' % 4U (kk pair 2j) of tile row
    // i' / 4U, i' = i % 64U; threads with equal i' load and store the same
    // value to the same slot (an unconditional store keeps the compiler from
    // sinking the prefetch load into a branch next to its use)
    const int si = tid % (64 * U);
    const int st_t = si / (4 * U), st_j = si % (4 * U);
    const float4 *st_row =
        reinterpret_cast<const float4 *>(X + ((size_t)k * nt + min(t0 + st_t, nt - 1)) * KKs);
    const float4 *fk = Ff + (size_t)k * (KKs / 8) * ncb * 64;
    // the lone output column xcol (if any) is summed on the vector ALU by every
    // wave (one broadcast 16-byte load per lane group and pair, negligible next
    // to the fragments); the last wave stores it.  Without one, Gx4 points at
    // valid memory and the sum is discarded, so the loop stays branch-free.
    const float4 *gxk = Gx4 + (xcol >= 0 ? (size_t)k * (KKs / 8) * 4 : 0);
    float2 accx = make_float2(0.f, 0.f);
    int cbi[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b)
        cbi[b] = min(wave * CB + b, ncb - 1);
    f32x4 accr[CB], acci[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
        accr[b] = f32x4{0.f, 0.f, 0.f, 0.f};
        acci[b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
#if LFRL_KARA
    f32x4 accs[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b)
        accs[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#endif
    auto a_load = [&](int grp) -> float4 {
        const int pg = min(p0 + grp * U + st_j / 4, p1 - 1);
        return st_row[4 * pg + st_j % 4];
    };
    auto a_store = [&](int grp, int buf, const float4 &v) {
        const int pg = p0 + grp * U + st_j / 4;
        const int kk = 8 * pg + 2 * (st_j % 4);
        const bool ok0 = pg < p1 && kk < KK, ok1 = pg < p1 && kk + 1 < KK;
        la[buf][st_j / 4][16 * (st_j % 4) + st_t] =
            make_float4(mask_f(v.x, ok0), mask_f(v.y, ok0), mask_f(v.z, ok1), mask_f(v.w, ok1));
    };
    auto b_load = [&](int grp, float4(&gb)[U][CB], float4(&gx)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = min(p0 + grp * U + u, p1 - 1);
#pragma unroll
            for (int b = 0; b < CB; ++b)
                gb[u][b] = fk[((size_t)p * ncb + cbi[b]) * 64 + lane];
            gx[u] = gxk[xcol >= 0 ? (size_t)p * 4 + kq : 0];
        }
    };
    auto column_group = [&](int buf, const float4(&gx)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float4 a = la[buf][u][lane], g = gx[u];
            accx.x = fmaf(a.x, g.x, fmaf(-a.y, g.y, fmaf(a.z, g.z, fmaf(-a.w, g.w, accx.x))));
            accx.y = fmaf(a.x, g.y, fmaf(a.y, g.x, fmaf(a.z, g.w, fmaf(a.w, g.z, accx.y))));
        }
    };
    auto compute_group = [&](int buf, const float4(&gb)[U][CB]) {
#if LFRL_KARA
        // three real products per complex product: accr = sum ar gr,
        // acci = sum ai gi, accs = sum (ar + ai)(gr + gi)
        // (a wave's surplus column blocks, which repeat its last one and are
        // not stored, skip their products: a wave-uniform branch)
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float4 a = la[buf][u][lane];
            const float s0 = a.x + a.y, s1 = a.z + a.w;
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                if (b > 0 && wave * CB + b >= ncb)
                    break;
                const float4 g = gb[u][b];
                accr[b] = mfma4(a.x, g.x, accr[b]);
                acci[b] = mfma4(a.y, g.y, acci[b]);
                accs[b] = mfma4(s0, g.x + g.y, accs[b]);
            }
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                if (b > 0 && wave * CB + b >= ncb)
                    break;
                const float4 g = gb[u][b];
                accr[b] = mfma4(a.z, g.z, accr[b]);
                acci[b] = mfma4(a.w, g.w, acci[b]);
                accs[b] = mfma4(s1, g.z + g.w, accs[b]);
            }
        }
        return;
#endif
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float4 a = la[buf][u][lane];
            // product-major order: consecutive MFMAs update different
            // accumulators (2 * CB independent chains)
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                accr[b] = mfma4(a.x, gb[u][b].x, accr[b]);
                acci[b] = mfma4(a.x, gb[u][b].y, acci[b]);
            }
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                accr[b] = mfma4(-a.y, gb[u][b].y, accr[b]);
                acci[b] = mfma4(a.y, gb[u][b].x, acci[b]);
            }
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                accr[b] = mfma4(a.z, gb[u][b].z, accr[b]);
                acci[b] = mfma4(a.z, gb[u][b].w, acci[b]);
            }
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                accr[b] = mfma4(-a.w, gb[u][b].w, accr[b]);
                acci[b] = mfma4(a.w, gb[u][b].z, acci[b]);
            }
        }
    };
    // Straight-line loop body: every group's loads are issued (clamped, so a
    // surplus group re-reads valid data) and every group is computed (surplus
    // pairs meet zeros in LDS).  A conditional prefetch would join paths with
    // different numbers of loads in flight, and the waits at the join would
    // then cover the prefetch too.  The scheduling barriers keep each
    // prefetch ahead of the products it is meant to overlap.
    float4 gb0[U][CB], gb1[U][CB], gx0[U], gx1[U];
    float4 av = a_load(0);
    b_load(0, gb0, gx0);
    a_store(0, 0, av);
    __syncthreads();
    for (int grp = 0; grp < ngroups; grp += 2) {
        av = a_load(grp + 1);
        b_load(grp + 1, gb1, gx1);
        __builtin_amdgcn_sched_barrier(0);
        compute_group(0, gb0);
        column_group(0, gx0);
        __builtin_amdgcn_sched_barrier(0);
        a_store(grp + 1, 1, av);
        __syncthreads();
        av = a_load(grp + 2);
        b_load(grp + 2, gb0, gx0);
        __builtin_amdgcn_sched_barrier(0);
        compute_group(1, gb1);
        column_group(1, gx1);
        __builtin_amdgcn_sched_barrier(0);
        a_store(grp + 2, 0, av);
        __syncthreads();
    }
#if LFRL_KARA
#pragma unroll
    for (int b = 0; b < CB; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float pr = accr[b][i], pi = acci[b][i];
            accr[b][i] = pr - pi;
            acci[b][i] = accs[b][i] - pr - pi;
        }
#endif
    // D[t][c]: lane holds tiles t0 + 4 * kq + i, column c of each block
    float2 *yk = Yp + ((size_t)s * nf + k) * nt * NN;
    // the lone column: lane (t, kq) holds tile t's partial over lane group kq
    accx.x += __shfl_xor(accx.x, 16, 64);
    accx.y += __shfl_xor(accx.y, 16, 64);
    accx.x += __shfl_xor(accx.x, 32, 64);
    accx.y += __shfl_xor(accx.y, 32, 64);
    if (xcol >= 0 && wave == (int)(blockDim.x >> 6) - 1 && kq == 0 && t0 + col < nt)
        yk[(size_t)(t0 + col) * NN + xcol] = accx;
#pragma unroll
    for (int b = 0; b < CB; ++b) {
        const int c = 16 * (wave * CB + b) + col;
        if (c >= NN || wave * CB + b >= ncb)
            continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int tt = t0 + 4 * kq + i;
            if (tt < nt)
                yk[(size_t)tt * NN + c] = make_float2(accr[b][i], acci[b][i]);
        }
    }
}

// Row stride (float2) of the staged image spectra rs[c][t] of the adjoint:
// 16 tiles plus one pad, so the coalesced staging writes spread over banks.
static constexpr int kRsStride = 17;

// Adjoint contraction for one frequency k and `ranges` ranges of kk, computed
// transposed so that tiles are the MFMA rows:
//   B[k][t][kk] = sum_c R[k][t][c] * conj(Gb[k][c][kk])
// A = R (16 tiles x NCp), staged once per block in LDS as rs[c][t] with
// coalesced loads along c and reused for every range; B = conj(H) from the Fb
// fragments (CB blocks of 16 kk per wave), with the same double-buffered,
// straight-line groups of U fragment pairs as the forward contraction.
template <int CB, int U>
__global__ __launch_bounds__(256) void k_contract_adj(const float4 *__restrict__ Fb,
                                                      const float2 *__restrict__ Rs,
                                                      float2 *__restrict__ B, int NN, int KK,
                                                      int KKs, int NCp, int nt, int ranges,
                                                      const int *__restrict__ skip, FreqMap fm,
                                                      const float2 *__restrict__ Hx, int xc,
                                                      int KKb, size_t osk, size_t ost)
{
    if (skip && *skip)
        return;
    extern __shared__ float2 rs[];  // [even number of groups of 8 * U rows][kRsStride]
    int k, by, tg;
    contraction_block(k, by, tg);
    k = unique_freq(k, fm);
    const int t0 = tg * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int nkb = (KK + 15) / 16;
    const int npairs = NCp / 8;
    const int ngroups = ((npairs + U - 1) / U + 1) / 2 * 2;  // even: see the loop
    const int ncl = ngroups * U * 8;
    // coalesced staging along c, in batches of loads issued before their
    // stores (clamped addresses; out-of-range values cleared by a bit mask)
    const int total = ncl * 16;
    for (int base = threadIdx.x; base < total; base += 8 * blockDim.x) {
        float2 v[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int idx = min(base + b * (int)blockDim.x, total - 1);
            const int tt = idx / ncl, c = idx % ncl;
            // rows past the fragments' NCp (a lone index xc among them) stay zero
            const bool ok = c < NN && c < NCp && t0 + tt < nt;
            const float2 x = Rs[((size_t)k * nt + min(t0 + tt, nt - 1)) * NN + min(c, NN - 1)];
            v[b] = make_float2(mask_f(x.x, ok), mask_f(x.y, ok));
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int idx = base + b * (int)blockDim.x;
            if (idx < total)
                rs[(idx % ncl) * kRsStride + idx / ncl] = v[b];
        }
    }
    __syncthreads();
    // the lone reduction index xc (if any) is not in the fragments: its
    // R values for this lane's four output rows
    float2 rx[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int tt = min(t0 + 4 * kq + i, nt - 1);
        rx[i] = xc >= 0 ? Rs[((size_t)k * nt + tt) * NN + xc] : make_float2(0.f, 0.f);
    }
    const float4 *fk = Fb + (size_t)k * npairs * nkb * 64;
    float2 *bk = B + (size_t)k * osk;   // rows of KKs: 128-byte aligned
    const int RB = nwaves * CB;  // column blocks per range (the packing's RB)
    for (int r = 0; r < ranges; ++r) {
        const int kb0 = ((by * ranges + r) * nwaves + wave) * CB;
        if (kb0 >= nkb)
            break;
        int kbi[CB];
        bool k_ok[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            k_ok[b] = kb0 + b < nkb;
            kbi[b] = k_ok[b] ? kb0 + b : nkb - 1;
        }
        f32x4 accr[CB], acci[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            accr[b] = f32x4{0.f, 0.f, 0.f, 0.f};
            acci[b] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
#if LFRL_KARA
        f32x4 accs[CB];
#pragma unroll
        for (int b = 0; b < CB; ++b)
            accs[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#endif
        float4 gb0[U][CB], gb1[U][CB];
        // pairs past the last read a valid fragment (clamped) that meets zeros in rs
        auto load_group = [&](int grp, float4(&gb)[U][CB]) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = min(grp * U + u, npairs - 1);
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    gb[u][b] = adj_load4(&fk[adj_frag(p, kbi[b], npairs, nkb, RB) * 64 + lane]);
            }
        };
        auto compute_group = [&](int grp, const float4(&gb)[U][CB]) {
#if LFRL_KARA
            // R conj(G) in three real products: accr = sum rr gr, acci = sum ri gi,
            // accs = sum (rr + ri)(gr - gi)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = 8 * (grp * U + u) + 2 * kq;
                const float2 a0 = rs[c * kRsStride + col], a1 = rs[(c + 1) * kRsStride + col];
                const float s0 = a0.x + a0.y, s1 = a1.x + a1.y;
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    const float4 g = gb[u][b];
                    accr[b] = mfma4(a0.x, g.x, accr[b]);
                    acci[b] = mfma4(a0.y, g.y, acci[b]);
                    accs[b] = mfma4(s0, g.x - g.y, accs[b]);
                }
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    const float4 g = gb[u][b];
                    accr[b] = mfma4(a1.x, g.z, accr[b]);
                    acci[b] = mfma4(a1.y, g.w, acci[b]);
                    accs[b] = mfma4(s1, g.z - g.w, accs[b]);
                }
            }
            return;
#endif
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = 8 * (grp * U + u) + 2 * kq;
                const float2 a0 = rs[c * kRsStride + col], a1 = rs[(c + 1) * kRsStride + col];
                // product-major order: consecutive MFMAs update different
                // accumulators (2 * CB independent chains)
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    accr[b] = mfma4(a0.x, gb[u][b].x, accr[b]);
                    acci[b] = mfma4(a0.y, gb[u][b].x, acci[b]);
                }
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    accr[b] = mfma4(a0.y, gb[u][b].y, accr[b]);
                    acci[b] = mfma4(-a0.x, gb[u][b].y, acci[b]);
                }
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    accr[b] = mfma4(a1.x, gb[u][b].z, accr[b]);
                    acci[b] = mfma4(a1.y, gb[u][b].z, acci[b]);
                }
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    accr[b] = mfma4(a1.y, gb[u][b].w, accr[b]);
                    acci[b] = mfma4(-a1.x, gb[u][b].w, acci[b]);
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
            compute_group(grp + 1, gb1);
            __builtin_amdgcn_sched_barrier(0);
        }
#if LFRL_KARA
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float pr = accr[b][i], pi = acci[b][i];
                accr[b][i] = pr + pi;
                acci[b][i] = accs[b][i] - pr + pi;
            }
#endif
        if (xc >= 0) {
            // + R[t][xc] conj(H[xc][kk]) on the vector ALU
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const float2 h = Hx[(size_t)k * KKb + 16 * kbi[b] + col];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    accr[b][i] = fmaf(rx[i].x, h.x, fmaf(rx[i].y, h.y, accr[b][i]));
                    acci[b][i] = fmaf(rx[i].y, h.x, fmaf(-rx[i].x, h.y, acci[b][i]));
                }
            }
        }
        // D[t][kk]: lane holds tiles t0 + 4 * kq + i, column kk of each block
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const int kk = 16 * kbi[b] + col;
            if (!k_ok[b] || kk >= KK)
                continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int tt = t0 + 4 * kq + i;
                if (tt < nt)
                    bk[(size_t)tt * ost + kk] = make_float2(accr[b][i], acci[b][i]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// metric kernels (sec. 2.2)
// ---------------------------------------------------------------------------

// Orthonormal DCT-II basis value c(f, n) cos((2x + 1) pi f / (2n)) (Eqs. 2-4),
// with the angle reduced exactly in integers before the cosine.
__device__ __forceinline__ double dct_basis(int f, int x, int n)
{
    const long long num = ((long long)(2 * x + 1) * f) % (4LL * n);
    const double c = (f == 0) ? sqrt(1.0 / n) : sqrt(2.0 / n);
    return c * cospi((double)num / (2.0 * n));
}

// tab[f][x] = c(f, n) cos((2x + 1) pi f / (2n)), f < nfreq, x < n (Eqs. 2-4).
__global__ void k_dct_table(double *__restrict__ tab, int n, int nfreq)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n * nfreq)
        tab[idx] = dct_basis(idx / n, idx % n, n);
}

// z maximum projection m[r][s] = max_j vol[j][r][s] (sec. 2.2, Fig. 2(a)) with
// per-block float64 partial sums of m^2 (Parseval: sum m^2 = ||F||_F^2).
__global__ void k_mip(const float *__restrict__ vol, int nz, size_t hw, float *__restrict__ mip,
                      double *__restrict__ n2p, const int *__restrict__ skip,
                      unsigned long long *__restrict__ zero, size_t nzero)
{
    // the multi-block spectral norm's exchange words (zero: no valid tag),
    // written through to device-coherent memory like the words themselves
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nzero;
         i += (size_t)gridDim.x * blockDim.x)
        __hip_atomic_store(zero + i, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (skip && *skip)
        return;
    __shared__ double red[256];
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    double sq = 0.0;
    if (i < hw) {
        // planes in batches of 8 loads (clamped: a repeated plane leaves the max)
        float m = vol[i];
        for (int j0 = 1; j0 < nz; j0 += 8) {
            float v[8];
#pragma unroll
            for (int b = 0; b < 8; ++b)
                v[b] = vol[(size_t)min(j0 + b, nz - 1) * hw + i];
#pragma unroll
            for (int b = 0; b < 8; ++b)
                m = fmaxf(m, v[b]);
        }
        mip[i] = m;
        sq = (double)m * (double)m;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        n2p[blockIdx.x] = red[0];
}

// Row transform over a chunk of image rows:
// T1[chunk][v][s] = sum_{r in chunk} C_H[v][r] m[r][s]  (float64).
__global__ void k_dct_rows(const float *__restrict__ mip, int H, int W,
                           const double *__restrict__ tabH, int nv, int rows_per_chunk,
                           double *__restrict__ T1)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int chunk = blockIdx.y;
    if (idx >= nv * W)
        return;
    const int v = idx / W, s = idx % W;
    const int r0 = chunk * rows_per_chunk, r1 = min(H, r0 + rows_per_chunk);
    const double *tv = tabH + (size_t)v * H;
    double acc = 0.0;
    int r = r0;
    for (; r + 8 <= r1; r += 8) {
        float m[8];
#pragma unroll
        for (int b = 0; b < 8; ++b)
            m[b] = mip[(size_t)(r + b) * W + s];
#pragma unroll
        for (int b = 0; b < 8; ++b)
            acc = fma(tv[r + b], (double)m[b], acc);
    }
    for (; r < r1; ++r)
        acc = fma(tv[r], (double)mip[(size_t)r * W + s], acc);
    T1[(size_t)chunk * nv * W + idx] = acc;
}

// Fold the row chunks into the first: T1[0][v][s] = sum_chunk T1[chunk][v][s].
__global__ void k_dct_fold(double *__restrict__ T1, int nchunks, int n)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n)
        return;
    double acc = T1[idx];
    for (int c0 = 1; c0 < nchunks; c0 += 8) {
        double v[8];
#pragma unroll
        for (int b = 0; b < 8; ++b)
            v[b] = T1[(size_t)min(c0 + b, nchunks - 1) * n + idx];
#pragma unroll
        for (int b = 0; b < 8; ++b)
            acc += (c0 + b < nchunks) ? v[b] : 0.0;
    }
    T1[idx] = acc;
}

// One wave per candidate coefficient (v, u):
// F[v][u] = sum_chunk sum_s T1[chunk][v][s] C_W[u][s] for (v, u) inside the
// region (LFRL_REGION_*: the triangle u / xs + v / ys < 1, the rectangle
// u < xs, v < ys, or everything); |F| is written, -1 marks coefficients outside.
__global__ void k_metric_coeffs(const double *__restrict__ T1, int nchunks, int nv, int nu, int W,
                                const double *__restrict__ tabW, double xs, double ys, int region,
                                double *__restrict__ Fabs)
{
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= nv * nu)
        return;
    const int v = wave / nu, u = wave % nu;
    const bool inside = region == LFRL_REGION_TRIANGLE ? ((double)u / xs + (double)v / ys) < 1.0
                        : region == LFRL_REGION_RECTANGLE ? ((double)u < xs && (double)v < ys)
                                                          : true;
    if (!inside) {
        if (lane == 0)
            Fabs[wave] = -1.0;
        return;
    }
    const double *tu = tabW + (size_t)u * W;
    double acc = 0.0;
    for (int s = lane; s < W; s += 64) {
        double t = 0.0;
        for (int c = 0; c < nchunks; ++c)
            t += T1[((size_t)c * nv + v) * W + s];
        acc = fma(t, tu[s], acc);
    }
    for (int off = 32; off > 0; off >>= 1)
        acc += __shfl_down(acc, off, 64);
    if (lane == 0)
        Fabs[wave] = fabs(acc);
}

// Whole-matrix DCT passes as tiled float64 matrix products:
//   C[m][n] = sum_k A[m][k] * B(k, n),  B(k, n) = BT ? B[n * ldb + k] : B[k * ldb + n],
// A row-major with leading dimension lda.  ABS: C holds |value| (coefficient
// magnitudes).  32 x 32 outputs per 256-thread block (2 x 2 per thread), k in
// slices of 32 staged in LDS; edges are zero-filled.
template <bool BT, bool ABS, typename TB>
__global__ __launch_bounds__(256) void k_dgemm32(const double *__restrict__ A, int lda,
                                                 const TB *__restrict__ B, int ldb, int M, int N,
                                                 int K, double *__restrict__ C, int ldc)
{
    __shared__ double As[32][33];  // [k][m]
    __shared__ double Bs[32][33];  // [k][n]
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int k0 = 0; k0 < K; k0 += 32) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int idx = tid + 256 * r;
            const int mm = idx / 32, kk = idx % 32;
            const int gm = m0 + mm, gk = k0 + kk;
            As[kk][mm] = (gm < M && gk < K) ? A[(size_t)gm * lda + gk] : 0.0;
            if (BT) {
                const int gn = n0 + mm;
                Bs[kk][mm] = (gn < N && gk < K) ? (double)B[(size_t)gn * ldb + gk] : 0.0;
            } else {
                const int gk2 = k0 + idx / 32, gn = n0 + idx % 32;
                Bs[idx / 32][idx % 32] =
                    (gn < N && gk2 < K) ? (double)B[(size_t)gk2 * ldb + gn] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < 32; ++kk) {
            const double a0 = As[kk][ty], a1 = As[kk][ty + 16];
            const double b0 = Bs[kk][tx], b1 = Bs[kk][tx + 16];
            acc[0][0] = fma(a0, b0, acc[0][0]);
            acc[0][1] = fma(a0, b1, acc[0][1]);
            acc[1][0] = fma(a1, b0, acc[1][0]);
            acc[1][1] = fma(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const int m = m0 + ty + 16 * i, n = n0 + tx + 16 * jj;
            if (m < M && n < N)
                C[(size_t)m * ldc + n] = ABS ? fabs(acc[i][jj]) : acc[i][jj];
        }
}

// Lane l's value of v, for every lane (l uniform).
__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Largest eigenvalue of the symmetric tridiagonal with diagonal al[0..k) and
// off-diagonal be[1..k), by multisection on one wave: Gershgorin bounds, then
// rounds in which lane l counts the eigenvalues below lo + (l + 1)(hi - lo)/65
// and the bracket shrinks to the two points around the largest one (about 9
// rounds to a width of two units in the last place).  The count is the number of sign changes of the
// characteristic polynomials of the leading submatrices (a Sturm sequence),
// formed without divisions on the matrix scaled to unit Gershgorin radius;
// a zero takes the sign opposite to its predecessor.  Row i of the matrix
// sits in lane i (k <= 64) and enters each Sturm step as scalar operands.
// Every lane of the calling wave takes part and returns the same value.
__device__ double wave_max_eig(const double *al, const double *be, int k, int lane)
{
    // lane i < k holds row i: its Gershgorin interval, then its scaled entries
    double glo = 1e308, ghi = -1e308;
    double ai = 0.0, bi = 0.0;
    if (lane < k) {
        ai = al[lane];
        bi = lane > 0 ? be[lane] : 0.0;
        const double r = fabs(bi) + (lane + 1 < k ? fabs(be[lane + 1]) : 0.0);
        glo = ai - r;
        ghi = ai + r;
    }
    for (int off = 32; off > 0; off >>= 1) {
        glo = fmin(glo, __shfl_xor(glo, off, 64));
        ghi = fmax(ghi, __shfl_xor(ghi, off, 64));
    }
    double lo = glo, hi = ghi;
    const double amax = fmax(fabs(lo), fabs(hi));
    if (!(amax > 0.0))
        return 0.0;  // the zero matrix
    const double sc = 1.0 / amax;
    const double as = ai * sc, b2s = (bi * sc) * (bi * sc);
    const double a0 = readlane_f64(as, 0);
    for (int round = 0; round < 40 && hi - lo > 4e-16 * fabs(hi); ++round) {
        const double step = (hi - lo) * (1.0 / 65.0);
        const double x = (lo + step * (double)(lane + 1)) * sc;
        double p0 = 1.0, p1 = a0 - x;
        // n1: p1 negative (a zero takes the opposite sign of its predecessor,
        // here p0 > 0); selects, no branches
        int n1 = p1 <= 0.0;
        int below = n1;
        // row i's entries come from lane i (uniform: scalar operands)
        auto sturm_step = [&](int i) {
            const double a = readlane_f64(as, i), b2 = readlane_f64(b2s, i);
            const double p2 = fma(a - x, p1, -b2 * p0);
            const int n2 = p2 == 0.0 ? 1 - n1 : (int)(p2 < 0.0);
            below += n2 ^ n1;
            p0 = p1;
            p1 = p2;
            n1 = n2;
        };
        int i = 1;
        for (; i + 4 <= k; i += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                sturm_step(i + u);
            // keep the pair in range (the ratio is what counts); on the scaled
            // matrix a step grows them at most threefold
            const double mag = fmax(fabs(p0), fabs(p1));
            const double f = mag > 1e150 ? 1e-150 : (mag < 1e-150 ? 1e150 : 1.0);
            p0 *= f;
            p1 *= f;
        }
        for (; i < k; ++i)
            sturm_step(i);
        // lanes whose point lies above every eigenvalue (monotone in the lane)
        const unsigned long long above = __ballot(below == k);
        const int fl = above ? __ffsll((long long)above) - 1 : 64;
        const double nlo = fl > 0 ? lo + step * (double)fl : lo;
        const double nhi = fl < 64 ? lo + step * (double)(fl + 1) : hi;
        if (!(nhi - nlo < hi - lo))
            break;  // the bracket no longer shrinks in double precision
        lo = nlo;
        hi = nhi;
    }
    return hi;
}

// Largest singular value squared of the h x w image m: the largest eigenvalue
// of A = B^T B, with B = m when w <= h and B = m^T otherwise (A of side
// n = min(h, w)), by Lanczos iteration in float64, in one block.  Step j:
// y = B v_j (one wave per 4 rows or one lane per column, in a fixed order),
// alpha_j = |y|^2 (= v_j . A v_j), w = B^T y - alpha_j v_j - beta_j v_{j-1},
// then once more orthogonalised against v_j and v_{j-1}; beta_{j+1} = |w|,
// v_{j+1} = w / beta_{j+1}.  No orthogonalisation against older vectors: the
// largest Ritz value converges to the largest eigenvalue all the same (a lost
// orthogonality only adds copies of converged values).  The largest eigenvalue
// theta of the tridiagonal (alpha, beta) comes from wave_max_eig.  Stops once
// theta grows by at most 1e-15 of itself, w vanishes (an invariant subspace:
// theta is exact), or after maxsteps steps.  v_0 is a fixed positive vector.
// Dynamic LDS: (3 n + max(h, w)) doubles.  *n2 = theta.
static constexpr int kLanczosMaxSteps = 48;
static_assert(kLanczosMaxSteps < 64, "wave_max_eig holds one tridiagonal row per lane");

__global__ __launch_bounds__(1024) void k_spectral_norm(const float *__restrict__ m, int H, int W,
                                                        int maxsteps, const int *__restrict__ skip,
                                                        double *__restrict__ n2)
{
    if (skip && *skip)
        return;
    extern __shared__ double sv[];
    __shared__ double red[2][16];
    __shared__ double al[kLanczosMaxSteps + 1], be[kLanczosMaxSteps + 1];
    __shared__ double theta_s;
    __shared__ int stop_s;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwave = nth >> 6;
    const bool tall = W <= H;             // A = m^T m (side W) or m m^T (side H)
    const int n = tall ? W : H, mo = tall ? H : W;
    double *x = sv, *xp = sv + n, *w = sv + 2 * n, *y = sv + 3 * n;  // v_j, v_{j-1}, w, B v_j
    // two block sums at once: wave sums by shuffles, then the waves in order
    auto block_sum2 = [&](double a, double c, double &ra, double &rc) {
        for (int off = 32; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            c += __shfl_xor(c, off, 64);
        }
        if (lane == 0) {
            red[0][wave] = a;
            red[1][wave] = c;
        }
        __syncthreads();
        ra = red[0][0];
        rc = red[1][0];
        for (int q = 1; q < nwave; ++q) {
            ra += red[0][q];
            rc += red[1][q];
        }
        __syncthreads();
    };
    // rows pass: out[r] = sum_s m[r][s] in[s], a wave per 4 rows at a time
    // (16 loads in flight per lane: the pass is bound by memory latency)
    auto rows_pass = [&](const double *in, double *out) {
        for (int r0 = 4 * wave; r0 < H; r0 += 4 * nwave) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int s0 = lane; s0 < W; s0 += 4 * 64) {
                float v4[4][4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        v4[q][b] = m[(size_t)min(r0 + q, H - 1) * W + min(s0 + 64 * b, W - 1)];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const double xv = s0 + 64 * b < W ? in[min(s0 + 64 * b, W - 1)] : 0.0;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        acc[q] = fma((double)v4[q][b], xv, acc[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double a = acc[q];
                for (int off = 32; off > 0; off >>= 1)
                    a += __shfl_down(a, off, 64);
                if (lane == 0 && r0 + q < H)
                    out[r0 + q] = a;
            }
        }
    };
    // columns pass: out[s] = sum_r m[r][s] in[r], one lane per column s < W,
    // rows in batches of 16 loads (in fixed order)
    auto cols_pass = [&](const double *in, double *out) {
        for (int s = tid; s < W; s += nth) {
            double acc = 0.0;
            int r = 0;
            for (; r + 16 <= H; r += 16) {
                float v16[16];
#pragma unroll
                for (int b = 0; b < 16; ++b)
                    v16[b] = m[(size_t)(r + b) * W + s];
#pragma unroll
                for (int b = 0; b < 16; ++b)
                    acc = fma((double)v16[b], in[r + b], acc);
            }
            for (; r < H; ++r)
                acc = fma((double)m[(size_t)r * W + s], in[r], acc);
            out[s] = acc;
        }
    };
    // v_0: fixed positive vector, unit length; v_{-1} = 0
    double c = 0.0;
    for (int i = tid; i < n; i += nth) {
        const double v = 1.0 + (double)((unsigned)(i + 1) * 2654435761u % 1024u) / 2048.0;
        x[i] = v;
        xp[i] = 0.0;
        c += v * v;
    }
    double n0, unused;
    block_sum2(c, 0.0, n0, unused);
    n0 = sqrt(n0);
    for (int i = tid; i < n; i += nth)
        x[i] /= n0;
    if (tid == 0) {
        theta_s = 0.0;
        stop_s = 0;
        be[0] = 0.0;
    }
    __syncthreads();
    const int steps = max(1, min(maxsteps, kLanczosMaxSteps));
    for (int j = 0; j < steps; ++j) {
        // y = B v_j; alpha_j = |y|^2
        if (tall)
            rows_pass(x, y);
        else
            cols_pass(x, y);
        __syncthreads();
        double a = 0.0;
        for (int i = tid; i < mo; i += nth)
            a += y[i] * y[i];
        double alpha;
        block_sum2(a, 0.0, alpha, unused);
        if (tid == 0)
            al[j] = alpha;
        __syncthreads();
        if (j + 1 == steps) {   // no room for another basis vector
            if (wave == 0) {
                const double th = wave_max_eig(al, be, j + 1, lane);
                if (lane == 0)
                    theta_s = th;
            }
            __syncthreads();
            break;
        }
        // w = B^T y - alpha v_j - beta_j v_{j-1}
        if (tall)
            cols_pass(y, w);
        else
            rows_pass(y, w);
        __syncthreads();
        const double bj = be[j];
        double c0 = 0.0, c1 = 0.0;
        for (int e = tid; e < n; e += nth) {
            const double t = w[e] - alpha * x[e] - bj * xp[e];
            w[e] = t;
            c0 = fma(t, x[e], c0);
            c1 = fma(t, xp[e], c1);
        }
        double d0, d1;
        block_sum2(c0, c1, d0, d1);
        double b2 = 0.0;
        for (int e = tid; e < n; e += nth) {
            const double t = w[e] - d0 * x[e] - d1 * xp[e];
            w[e] = t;
            b2 = fma(t, t, b2);
        }
        double bb;
        block_sum2(b2, 0.0, bb, unused);
        const double beta = sqrt(bb);
        if (wave == 0) {
            const double th = wave_max_eig(al, be, j + 1, lane);
            // converged: the largest Ritz value no longer grows, or w vanished
            // (the Krylov space is invariant and th is exact)
            if (lane == 0) {
                if ((j > 0 && th - theta_s <= 1e-15 * th) || !(beta > 1e-14 * th))
                    stop_s = 1;
                theta_s = th;
                be[j + 1] = beta;
            }
        }
        __syncthreads();
        if (stop_s)
            break;
        // v_{j-1} = v_j, v_{j+1} = w / beta
        for (int e = tid; e < n; e += nth) {
            xp[e] = x[e];
            x[e] = w[e] / beta;
        }
        __syncthreads();
    }
    if (tid == 0)
        *n2 = theta_s;
}

// The same Lanczos iteration over many blocks, for images that one block
// would stream too slowly at each step.  A = m^T m throughout (vectors of
// length W).  Block b keeps rows [b rpb, (b + 1) rpb) of m in LDS and forms,
// for its rows, y_r = m_r . v_j (thread (r, s) sums the columns s, s + nseg,
// ... of row r, then the nseg pieces are added in order), its share
// sum_r y_r^2 of alpha_j and its partial sum_r y_r m_r of A v_j (a thread per
// column, rows in order): no cross-lane reductions.  One grid-wide exchange
// per step: every block then adds all partials in block order and carries out
// the rest of the step (the recurrence, beta, the Ritz value, the stop test)
// on identical data, so all blocks reach the same decisions.
//
// The exchange carries its own validity: each partial (a double) travels as
// two 64-bit words, each holding 32 bits of the value and the tag j + 1 of the
// step, written and read with device-coherent 64-bit accesses (single-copy
// atomic), so a reader polls each word until it carries the expected tag and
// no fence or counter is needed.  The words are zeroed by k_mip before every
// call (a zero tag never matches) and alternate between two buffers by step
// parity (a block writes step j + 2 only after reading every block's step
// j + 1, which they wrote after reading step j).  All blocks must be resident
// at once (few blocks, one per CU at most by their LDS); a wait that does not
// end within a bounded number of polls raises a failure flag that every
// block's waits also watch, and the result is then NaN instead of a hang.
// ws (64-bit words): [0] failure flag, [64 ...] the partials
//     [2][nb][W + 1][2] (zeroed by k_mip: spectral_mb_words(nb, W) words).
// Dynamic LDS: (3 W + spectral_mb_pieces(rpb, W) + rpb) doubles + rpb W floats.
static constexpr unsigned kSpinLimit = 1u << 18;

__host__ __device__ __forceinline__ int spectral_mb_segs(int rpb, int W)
{
    return max(1, min(W, 1024 / max(rpb, 1)));
}
__host__ __device__ __forceinline__ int spectral_mb_pieces(int rpb, int W)
{
    return rpb * spectral_mb_segs(rpb, W);
}
__host__ __device__ __forceinline__ size_t spectral_mb_words(int nb, int W)
{
    return 64 + (size_t)4 * nb * (W + 1);
}

__global__ __launch_bounds__(1024) void k_spectral_norm_mb(const float *__restrict__ m, int H, int W,
                                                           int rpb, int maxsteps,
                                                           unsigned long long *ws,
                                                           const int *__restrict__ skip,
                                                           double *__restrict__ n2)
{
    if (skip && *skip)
        return;
    extern __shared__ double lds[];
    __shared__ double red3[3][16];
    __shared__ double ashare_s;
    __shared__ double al[kLanczosMaxSteps + 1], be[kLanczosMaxSteps + 1];
    __shared__ double theta_s, alpha_s;
    __shared__ int stop_s, fail_s;
    const int nb = gridDim.x, b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    unsigned long long *fail_g = ws;
    unsigned long long *part = ws + 64;
    const int nseg = spectral_mb_segs(rpb, W);
    double *v = lds, *vp = lds + W, *wv = lds + 2 * W;
    double *py = lds + 3 * W;                        // [rpb][nseg] pieces of y
    double *yr = py + (size_t)rpb * nseg;            // [rpb]
    float *ms = reinterpret_cast<float *>(yr + rpb);  // [rpb][W]
    const int r0 = b * rpb, nr = max(0, min(H, r0 + rpb) - r0);
    for (size_t i = tid; i < (size_t)nr * W; i += 1024)
        ms[i] = m[(size_t)r0 * W + i];
    // three block sums at once: wave sums by shuffles, then the waves in order
    auto block_sum3 = [&](double a, double c, double e, double &ra, double &rc, double &re) {
        for (int off = 32; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            c += __shfl_xor(c, off, 64);
            e += __shfl_xor(e, off, 64);
        }
        if (lane == 0) {
            red3[0][wave] = a;
            red3[1][wave] = c;
            red3[2][wave] = e;
        }
        __syncthreads();
        ra = red3[0][0];
        rc = red3[1][0];
        re = red3[2][0];
        for (int q = 1; q < 16; ++q) {
            ra += red3[0][q];
            rc += red3[1][q];
            re += red3[2][q];
        }
        __syncthreads();
    };
    // v_0: the fixed positive vector of the one-block kernel, unit length
    double c = 0.0;
    for (int i = tid; i < W; i += 1024) {
        const double x = 1.0 + (double)((unsigned)(i + 1) * 2654435761u % 1024u) / 2048.0;
        v[i] = x;
        vp[i] = 0.0;
        c += x * x;
    }
    double n0, unused, unused2;
    block_sum3(c, 0.0, 0.0, n0, unused, unused2);
    n0 = sqrt(n0);
    for (int i = tid; i < W; i += 1024)
        v[i] /= n0;
    if (tid == 0) {
        theta_s = 0.0;
        stop_s = 0;
        fail_s = 0;
        be[0] = 0.0;
    }
    __syncthreads();
    const int steps = max(1, min(maxsteps, kLanczosMaxSteps));
    for (int j = 0; j < steps; ++j) {
        const unsigned long long tag = (unsigned long long)(j + 1) << 32;
        // y_r in pieces: thread (r, s) over the columns s, s + nseg, ...
        // (four running sums, four loads in flight, added in order)
        for (int it = tid; it < nr * nseg; it += 1024) {
            const int r = it / nseg, sg = it % nseg;
            const float *row = ms + (size_t)r * W;
            double d[4] = {0.0, 0.0, 0.0, 0.0};
            int cc = sg;
            for (; cc + 3 * nseg < W; cc += 4 * nseg) {
                float mv[4];
                double vv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    mv[q] = row[cc + q * nseg];
                    vv[q] = v[cc + q * nseg];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    d[q] = fma((double)mv[q], vv[q], d[q]);
            }
            for (int q = 0; cc < W; cc += nseg, ++q)
                d[q] = fma((double)row[cc], v[cc], d[q]);
            py[it] = (d[0] + d[1]) + (d[2] + d[3]);
        }
        __syncthreads();
        for (int r = tid; r < nr; r += 1024) {
            const double *pr = py + (size_t)r * nseg;
            double y = 0.0;
            int sg = 0;
            for (; sg + 8 <= nseg; sg += 8) {
                double t[8];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    t[q] = pr[sg + q];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    y += t[q];
            }
            for (; sg < nseg; ++sg)
                y += pr[sg];
            yr[r] = y;
        }
        __syncthreads();
        // alpha's share sum_r y_r^2 by the last wave (rows lane, lane + 64, ...,
        // then a butterfly), the other waves go on with their columns
        if (wave == 15) {
            double a2 = 0.0;
            for (int r = lane; r < nr; r += 64)
                a2 = fma(yr[r], yr[r], a2);
            for (int off = 32; off > 0; off >>= 1)
                a2 += __shfl_xor(a2, off, 64);
            if (lane == 0)
                ashare_s = a2;
        }
        // partial A v_j = sum_r y_r m_r: a thread per column, rows in order
        // (four running sums over r mod 4, eight rows in flight); sent with
        // alpha's share as tagged words
        unsigned long long *pb = part + ((size_t)(j & 1) * nb + b) * (W + 1) * 2;
        // (the share's words go last, from the thread of column W, after a
        // barrier that publishes it)
        for (int cc = tid; cc < W; cc += 1024) {
            double val;
            {
                double d[4] = {0.0, 0.0, 0.0, 0.0};
                int r = 0;
                for (; r + 8 <= nr; r += 8) {
                    float mv[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        mv[q] = ms[(size_t)(r + q) * W + cc];
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        d[q & 3] = fma(yr[r + q], (double)mv[q], d[q & 3]);
                }
                for (; r < nr; ++r)
                    d[r & 3] = fma(yr[r], (double)ms[(size_t)r * W + cc], d[r & 3]);
                val = (d[0] + d[1]) + (d[2] + d[3]);
            }
            const unsigned long long bits = (unsigned long long)__double_as_longlong(val);
            __hip_atomic_store(pb + 2 * cc, tag | (bits & 0xffffffffull), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(pb + 2 * cc + 1, tag | (bits >> 32), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (tid == 0) {
            const unsigned long long bits = (unsigned long long)__double_as_longlong(ashare_s);
            __hip_atomic_store(pb + 2 * W, tag | (bits & 0xffffffffull), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(pb + 2 * W + 1, tag | (bits >> 32), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        // A v_j and alpha_j: every block's words for this thread's column, in
        // block order (batches of 16 blocks, 32 loads in flight; a word with an
        // older tag is read again until it carries this step's)
        const unsigned long long *pj = part + (size_t)(j & 1) * nb * (W + 1) * 2;
        unsigned spins = 0;
        bool failed = false;
        for (int e = tid; e <= W; e += 1024) {
            double a = 0.0;
            for (int q0 = 0; q0 < nb; q0 += 16) {
                unsigned long long wd[16][2];
#pragma unroll
                for (int q = 0; q < 16; ++q)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        wd[q][h] = __hip_atomic_load(
                            pj + ((size_t)min(q0 + q, nb - 1) * (W + 1) + e) * 2 + h,
                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    if (q0 + q >= nb)
                        continue;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        while ((wd[q][h] & 0xffffffff00000000ull) != tag && !failed) {
                            if (++spins >= kSpinLimit ||
                                ((spins & 255) == 0 &&
                                 __hip_atomic_load(fail_g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                                __hip_atomic_store(fail_g, 1ull, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                                failed = true;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                            wd[q][h] = __hip_atomic_load(
                                pj + ((size_t)(q0 + q) * (W + 1) + e) * 2 + h, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                    const unsigned long long bits =
                        (wd[q][0] & 0xffffffffull) | ((wd[q][1] & 0xffffffffull) << 32);
                    a += __longlong_as_double((long long)bits);
                }
            }
            if (e < W)
                wv[e] = a;
            else
                alpha_s = a;
        }
        if (failed)
            fail_s = 1;
        __syncthreads();
        if (fail_s)
            break;
        const double alpha = alpha_s;
        if (tid == 0)
            al[j] = alpha;
        __syncthreads();
        if (j + 1 == steps) {  // no room for another basis vector
            if (wave == 0) {
                const double th = wave_max_eig(al, be, j + 1, lane);
                if (lane == 0)
                    theta_s = th;
            }
            __syncthreads();
            break;
        }
        // t = A v_j - alpha v_j - beta_j v_{j-1}, then w = t - (t.v_j) v_j -
        // (t.v_{j-1}) v_{j-1}; |w|^2 = |t|^2 - (t.v_j)^2 - (t.v_{j-1})^2 for
        // orthonormal v_j, v_{j-1} (one block sum for all three); where that
        // difference is small against |t|^2 it is summed directly instead
        const double bj = be[j];
        double c0 = 0.0, c1 = 0.0, tt = 0.0;
        for (int e = tid; e < W; e += 1024) {
            const double t = wv[e] - alpha * v[e] - bj * vp[e];
            wv[e] = t;
            c0 = fma(t, v[e], c0);
            c1 = fma(t, vp[e], c1);
            tt = fma(t, t, tt);
        }
        double d0, d1, t2;
        block_sum3(c0, c1, tt, d0, d1, t2);
        double bb = t2 - d0 * d0 - d1 * d1;
        const bool direct = !(bb > 1e-6 * t2);
        double b2 = 0.0;
        for (int e = tid; e < W; e += 1024) {
            const double t = wv[e] - d0 * v[e] - d1 * vp[e];
            wv[e] = t;
            b2 = fma(t, t, b2);
        }
        if (direct)  // block-uniform
            block_sum3(b2, 0.0, 0.0, bb, unused, unused2);
        const double beta = sqrt(bb);
        if (wave == 0) {
            const double th = wave_max_eig(al, be, j + 1, lane);
            if (lane == 0) {
                if ((j > 0 && th - theta_s <= 1e-15 * th) || !(beta > 1e-14 * th))
                    stop_s = 1;
                theta_s = th;
                be[j + 1] = beta;
            }
        }
        __syncthreads();
        if (stop_s)
            break;
        for (int e = tid; e < W; e += 1024) {
            vp[e] = v[e];
            v[e] = wv[e] / beta;
        }
        __syncthreads();
    }
    if (b == 0 && tid == 0)
        *n2 = fail_s ? __builtin_nan("") : theta_s;
}

// Per-block partial sums of |F|^2 over the coefficients inside the region
// (Fabs >= 0), for the region norm of a large coefficient set.
__global__ void k_sq_partial(const double *__restrict__ Fabs, int ncoef, double *__restrict__ part)
{
    __shared__ double red[256];
    double a = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncoef; i += gridDim.x * blockDim.x) {
        const double f = Fabs[i];
        if (f > 0.0)
            a += f * f;
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = red[0];
}

// Per-block partial sums of p log2 p, p = |F| / n over the coefficients inside
// the region.  Every block forms n^2 from the same partial sums (n2src,
// n2count) in the same order, so all blocks divide by the same n.
__global__ void k_entropy_partial(const double *__restrict__ n2src, int n2count,
                                  const double *__restrict__ Fabs, int ncoef,
                                  double *__restrict__ part)
{
    __shared__ double red[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n2count; i += blockDim.x)
        a += n2src[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    const double n = sqrt(red[0]);
    __syncthreads();
    double e = 0.0;
    if (n > 0.0) {
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncoef;
             i += gridDim.x * blockDim.x) {
            const double f = Fabs[i];
            if (f > 0.0) {
                const double p = f / n;
                e += p * log2(p);
            }
        }
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = red[0];
}

// Device-side Richardson-Lucy stop state.
struct StopState {
    double best_e;
    double prev_e;
    double sum_img;
    int best_k;
    int run;
    int stopped;
    int stop_k;
    int copy_flag;
    int iter;
};

// Record iteration k's metric e in the stop state (one thread): trace[k-1] = e,
// the best iterate (ties: later) and the stop flag, raised after `patience`
// consecutive strict decreases of the mean of the last `window` values (the
// trace holds e_1 .. e_k).
__device__ void record_metric(double e, StopState *st, double *trace, int k, int patience,
                              int window)
{
    trace[k - 1] = e;
    st->iter = k;
    if (k > window) {
        // means of e_{k-window+1..k} and e_{k-window..k-1}, oldest first
        double s1 = 0.0, s0 = 0.0;
        for (int i = k - window; i < k; ++i)
            s1 += trace[i];
        for (int i = k - 1 - window; i < k - 1; ++i)
            s0 += trace[i];
        st->run = (s1 / window < s0 / window) ? st->run + 1 : 0;
    }
    st->copy_flag = (k == 1 || e >= st->best_e) ? 1 : 0;
    if (st->copy_flag) {
        st->best_e = e;
        st->best_k = k;
    }
    st->prev_e = e;
    if (!st->stopped && st->run >= patience) {
        st->stopped = 1;
        st->stop_k = k;
    }
}

// Final entropy (Eq. 12) and stop rule.  Single block.  The norm is the
// Frobenius norm of the whole matrix (from Parseval's partial sums n2p), the
// spectral norm (its square in n2p[n2count], from k_spectral_norm) or the
// Frobenius norm of
// the coefficients inside the region (norm == LFRL_NORM_REGION), and the
// prefactor 1 / area.  out[0] = e.  When st != nullptr, iteration `k` is
// recorded: trace[k-1] = e, the best iterate is tracked (ties: later) and the
// stop flag raised after `patience` consecutive strict decreases of the mean
// of the last `window` values (trace must then hold e_1 .. e_k).
//
// With ent_part != nullptr the entropy sum arrives as nent block partials of
// k_entropy_partial instead (large coefficient sets) and Fabs is not read.
__global__ void k_metric_final(const double *__restrict__ n2p, int n2count,
                               const double *__restrict__ Fabs, int ncoef, int norm, double area,
                               double *__restrict__ out, StopState *st, double *trace, int k,
                               int patience, int window, const double *__restrict__ ent_part,
                               int nent, const int *skip)
{
    // a frame that stopped before this iteration records nothing (block-uniform;
    // skip points into *st, which only thread 0 writes, after the barriers)
    if (skip && *skip)
        return;
    __shared__ double red[256];
    double a = 0.0;
    if (ent_part) {
        a = 0.0;
    } else if (norm == LFRL_NORM_SPECTRAL) {
        a = threadIdx.x == 0 ? n2p[n2count] : 0.0;  // the Lanczos value
    } else if (norm == LFRL_NORM_REGION) {
        for (int i = threadIdx.x; i < ncoef; i += blockDim.x) {
            const double f = Fabs[i];
            if (f > 0.0)
                a += f * f;
        }
    } else {
        for (int i = threadIdx.x; i < n2count; i += blockDim.x)
            a += n2p[i];
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    const double n = ent_part ? 1.0 : sqrt(red[0]);
    __syncthreads();
    double e_part = 0.0;
    if (ent_part) {
        for (int i = threadIdx.x; i < nent; i += blockDim.x)
            e_part += ent_part[i];
    } else if (n > 0.0) {
        for (int i = threadIdx.x; i < ncoef; i += blockDim.x) {
            const double f = Fabs[i];
            if (f > 0.0) {
                const double p = f / n;
                e_part += p * log2(p);
            }
        }
    }
    red[threadIdx.x] = e_part;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double e = (n > 0.0 && red[0] != 0.0) ? -(1.0 / area) * red[0] : 0.0;
        out[0] = e;
        if (st)
            record_metric(e, st, trace, k, patience, window);
    }
}

// The whole metric of a small image in one block (run_metric's limits keep
// every buffer in LDS): z maximum projection and Parseval sum, the row
// transform for the nv candidate rows, the nv x nu candidate coefficients of
// the triangle or rectangle, the norm, the entropy and the stop rule; then,
// when the iterate is the best so far, its copy into best (nvox floats; best ==
// nullptr: no copy).  Dynamic LDS: nv * w + nv * nu doubles, then h * w floats.
__global__ __launch_bounds__(1024) void k_metric_small(
    const float *__restrict__ vol, int nz, int H, int W, const double *__restrict__ tabH,
    const double *__restrict__ tabW, int nv, int nu, double xs, double ys, int region, int norm,
    double area, double *__restrict__ out, StopState *st, double *trace, int k, int patience,
    int window, float *__restrict__ best, size_t nvox, const int *skip)
{
    if (skip && *skip)
        return;
    extern __shared__ double sm[];
    __shared__ double red[1024];
    __shared__ int flag;
    const int hw = H * W;
    double *T1 = sm;                                    // [nv][W]
    double *F = T1 + (size_t)nv * W;                    // [nv][nu]
    float *m = reinterpret_cast<float *>(F + (size_t)nv * nu);  // [H][W]
    const int tid = threadIdx.x, nth = blockDim.x;
    auto block_sum = [&](double a) -> double {
        red[tid] = a;
        __syncthreads();
        for (int off = nth / 2; off > 0; off >>= 1) {
            if (tid < off)
                red[tid] += red[tid + off];
            __syncthreads();
        }
        const double r = red[0];
        __syncthreads();
        return r;
    };
    double sq = 0.0;
    for (int i = tid; i < hw; i += nth) {
        float v = vol[i];
        for (int j = 1; j < nz; ++j)
            v = fmaxf(v, vol[(size_t)j * hw + i]);
        m[i] = v;
        sq += (double)v * (double)v;
    }
    const double n2 = block_sum(sq);  // its barriers also publish m
    for (int idx = tid; idx < nv * W; idx += nth) {
        const int v = idx / W, s = idx % W;
        const double *tv = tabH + (size_t)v * H;
        double acc = 0.0;
        for (int r = 0; r < H; ++r)
            acc = fma(tv[r], (double)m[r * W + s], acc);
        T1[idx] = acc;
    }
    __syncthreads();
    for (int c = tid; c < nv * nu; c += nth) {
        const int v = c / nu, u = c % nu;
        const bool inside = region == LFRL_REGION_TRIANGLE
                                ? ((double)u / xs + (double)v / ys) < 1.0
                                : ((double)u < xs && (double)v < ys);
        double f = -1.0;
        if (inside) {
            const double *tu = tabW + (size_t)u * W;
            double acc = 0.0;
            for (int s = 0; s < W; ++s)
                acc = fma(T1[v * W + s], tu[s], acc);
            f = fabs(acc);
        }
        F[c] = f;
    }
    __syncthreads();
    double nn = n2;
    if (norm == LFRL_NORM_REGION) {
        double a = 0.0;
        for (int c = tid; c < nv * nu; c += nth)
            if (F[c] > 0.0)
                a += F[c] * F[c];
        nn = block_sum(a);
    }
    const double n = sqrt(nn);
    double ep = 0.0;
    if (n > 0.0)
        for (int c = tid; c < nv * nu; c += nth) {
            const double f = F[c];
            if (f > 0.0) {
                const double p = f / n;
                ep += p * log2(p);
            }
        }
    const double es = block_sum(ep);
    if (tid == 0) {
        const double e = (n > 0.0 && es != 0.0) ? -(1.0 / area) * es : 0.0;
        out[0] = e;
        flag = 0;
        if (st) {
            record_metric(e, st, trace, k, patience, window);
            flag = st->copy_flag;
        }
    }
    __syncthreads();
    if (best && flag)
        for (size_t i = tid; i < nvox; i += nth)
            best[i] = vol[i];
}

__global__ void k_state_reset(StopState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->best_e = -1.0e300;
        st->prev_e = 0.0;
        st->sum_img = 0.0;
        st->best_k = 0;
        st->run = 0;
        st->stopped = 0;
        st->stop_k = 0;
        st->copy_flag = 0;
        st->iter = 0;
    }
}

// dst = src when the stop state says the current iterate is the best so far.
__global__ void k_cond_copy(const StopState *__restrict__ st, const float *__restrict__ src,
                            float *__restrict__ dst, size_t n)
{
    if (!st->copy_flag)
        return;
    const size_t n4 = n / 4;
    const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const float4 *s4 = reinterpret_cast<const float4 *>(src);
    float4 *d4 = reinterpret_cast<float4 *>(dst);
    for (size_t i = tid; i < n4; i += stride)
        d4[i] = s4[i];
    for (size_t i = n4 * 4 + tid; i < n; i += stride)
        dst[i] = src[i];
}

__global__ void k_zero_u32n(unsigned *__restrict__ p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_fill(float *__restrict__ p, size_t n, float v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Per-block float64 partials of sum(a * b) (b == nullptr: sum(a)).
__global__ void k_dot_partial(const float *__restrict__ a, const float *__restrict__ b, size_t n,
                              double *__restrict__ part)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        acc += b ? (double)a[i] * (double)b[i] : (double)a[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = red[0];
}

// Fixed-order sum of the dot partials.  which = 0: store the image sum in the
// stop state; which = 1: record the flux deviation <c, x^k> / sum(img) - 1.
__global__ void k_dot_final(const double *__restrict__ part, int nparts, StopState *st,
                            double *flux_trace, int k, int which)
{
    __shared__ double red[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x)
        a += part[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (which == 0)
            st->sum_img = red[0];
        else
            flux_trace[k - 1] = (st->sum_img != 0.0) ? red[0] / st->sum_img - 1.0 : 0.0;
    }
}

// ---------------------------------------------------------------------------
// FFT tile kernels: supported sizes and dispatch
// ---------------------------------------------------------------------------
// Tile sides with an FFT kernel (7-smooth, register-resident).  Other sides use
// the direct-sum DFT kernels above.
#define LFRL_FFT_Q_LIST(X) \
    X(8) X(9) X(10) X(12) X(14) X(15) X(16) X(18) X(20) X(21) X(24) X(25) X(27) X(28) X(30) \
    X(32) X(35) X(36) X(40) X(42) X(45) X(48)

static bool fft_supported(int Q)
{
    switch (Q) {
#define LFRL_CASE(q) case q:
        LFRL_FFT_Q_LIST(LFRL_CASE)
#undef LFRL_CASE
        return true;
    default:
        return false;
    }
}

// LDS of the forward tile DFT: the PSF mode stages its input tile; the planes
// mode needs only the half spectrum Z and twiddles (the column magnitudes for
// the row maxima reuse Z).
static size_t lds_r2c_fft(const Geo &g)
{
    const size_t a = (size_t)g.Q * g.Q * g.N * 4, b = (size_t)g.Q * g.QH * g.N * 8;
    return std::max(a, b) + (size_t)g.Q * 8;
}

static size_t lds_r2c_fft_planes(const Geo &g)
{
    return (size_t)g.Q * g.QH * g.N * 8 + (size_t)g.Q * 8;
}

static size_t lds_c2r_fft(const Geo &g)
{
    // twiddles, the T valid rows of the column inverse, the output tile
    return (size_t)g.Q * 8 + (size_t)g.T * g.QH * g.N * 8 + (size_t)g.T * g.T * g.N * 4;
}

static int round64(int v)
{
    return (v + 63) / 64 * 64;
}

// LDS of the inverse transform's staged epilogue inputs (two arrays of the
// tile's output pixels, rounded up to whole wave loads).
static size_t c2r_stage_bytes(const Geo &g)
{
    return (size_t)2 * round64(g.T * g.T * g.N) * 4;
}

// Stage the epilogue inputs when the larger LDS still admits as many blocks
// per CU (of 160 KiB, up to the four that the registers allow) as without.
static bool c2r_stage_fits(const Geo &g, size_t lds_max)
{
    const size_t cu = 160 * 1024, base = lds_c2r_fft(g), st = base + c2r_stage_bytes(g);
    return st <= lds_max && cu / st >= std::min<size_t>(4, cu / base);
}

// One thread per row pair / column of a tile; the kernels are built for at
// most kFftMaxThreads threads per block (which leaves 256 VGPRs per thread).
static constexpr int kFftMaxThreads = 512;

static int threads_r2c_fft(const Geo &g)
{
    return round64(std::max((g.Q * g.N + 1) / 2, g.QH * g.N));
}

static int threads_c2r_fft(const Geo &g)
{
    return round64(std::max(g.QH * g.N, (g.T * g.N + 1) / 2));
}

static bool fft_usable(const Geo &g, size_t lds_max)
{
    return fft_supported(g.Q) && threads_r2c_fft(g) <= kFftMaxThreads &&
           threads_c2r_fft(g) <= kFftMaxThreads && lds_r2c_fft(g) <= lds_max &&
           lds_c2r_fft(g) <= lds_max;
}

// The dynamic-LDS limit of a kernel holds for every later launch on the
// device, while plans of one tile side (and different Nnum) need different
// amounts: the limit is only ever raised (per kernel and device), so a plan
// built later never lowers what an earlier one launches with.
static size_t lds_limit();

// (A fixed table, so that no call allocates host memory either; should it
// ever fill, the limit is set to the whole LDS of a workgroup, which is never
// too low.)
static void raise_lds_attr(const void *fn, size_t lds)
{
    struct Entry {
        const void *fn;
        int dev;
        size_t lds;
    };
    static constexpr int kEntries = 1024;
    static std::mutex mu;
    static Entry set[kEntries];
    static int nset = 0;
    int dev = -1;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < nset; ++i) {
        Entry &e = set[i];
        if (e.fn == fn && e.dev == dev) {
            if (lds > e.lds) {
                (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                e.lds = lds;
            }
            return;
        }
    }
    if (nset == kEntries) {
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)std::max(lds, lds_limit()));
        return;
    }
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    set[nset++] = {fn, dev, lds};
}

static void set_fft_lds_attrs(int Q, size_t lds)
{
    switch (Q) {
#define LFRL_CASE(q)                                                                        \
    case q:                                                                                 \
        raise_lds_attr((const void *)k_r2c_fft<q>, lds);                                     \
        raise_lds_attr((const void *)k_c2r_fft<q>, lds);                                     \
        break;
        LFRL_FFT_Q_LIST(LFRL_CASE)
#undef LFRL_CASE
    default:
        break;
    }
}

static void launch_r2c_fft(int Q, dim3 grid, int block, size_t lds, hipStream_t st, int mode,
                           const TileBatch &batch, const float *src, int N, int T, int hD, int nt,
                           int KKo, int K, int c0, int KK, float2 *out, const float2 *tw,
                           unsigned *rowmax = nullptr)
{
    switch (Q) {
#define LFRL_CASE(q)                                                                        \
    case q:                                                                                 \
        hipLaunchKernelGGL(k_r2c_fft<q>, grid, dim3(block), lds, st, mode, batch, src, N, T, \
                           hD, nt, KKo, K, c0, KK, out, tw, rowmax);                         \
        break;
        LFRL_FFT_Q_LIST(LFRL_CASE)
#undef LFRL_CASE
    default:
        break;
    }
}

static void launch_c2r_fft(int Q, dim3 grid, int block, size_t lds, hipStream_t st,
                           const TileBatch &batch, const float2 *spec, size_t split_stride,
                           int nsplit, size_t sk, size_t stile, size_t sc, int N, int planes,
                           int T, int hD, const float2 *tw, int stage)
{
    switch (Q) {
#define LFRL_CASE(q)                                                                        \
    case q:                                                                                 \
        hipLaunchKernelGGL(k_c2r_fft<q>, grid, dim3(block), lds, st, batch, spec,            \
                           split_stride, nsplit, sk, stile, sc, N, planes, T, hD, tw, stage); \
        break;
        LFRL_FFT_Q_LIST(LFRL_CASE)
#undef LFRL_CASE
    default:
        break;
    }
}

// ---------------------------------------------------------------------------
// weakly observed voxels
// ---------------------------------------------------------------------------
// A voxel whose PSF footprint barely overlaps the image has a tiny sensitivity
// c = A^T 1, and the update x * (A^T rho) / c divides two small numbers whose
// float32 tile-DFT values carry absolute round-off of the image's scale.  Such
// voxels (c below a small fraction of the largest c) are listed once per image
// size and their window sums are evaluated directly in float64 instead.

// Per-block maxima of max(a, 0).
__global__ void k_max_partial(const float *__restrict__ a, size_t n, float *__restrict__ part)
{
    __shared__ float red[256];
    float m = 0.f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        m = fmaxf(m, a[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = red[0];
}

__global__ void k_max_final(const float *__restrict__ part, int nparts, float *__restrict__ out,
                            unsigned *__restrict__ count)
{
    __shared__ float red[256];
    float m = 0.f;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x)
        m = fmaxf(m, part[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0];
        *count = 0u;
    }
}

// Append voxels with sens < thr_rel * max to `list` (order not significant);
// *count ends as the number found, which may exceed cap (extra entries dropped).
__global__ void k_weak_select(const float *__restrict__ sens, size_t n,
                              const float *__restrict__ cmax, float thr_rel,
                              unsigned *__restrict__ list, unsigned *__restrict__ count,
                              unsigned cap)
{
    const float thr = thr_rel * cmax[0];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        if (sens[i] < thr) {
            const unsigned slot = atomicAdd(count, 1u);
            if (slot < cap)
                list[slot] = (unsigned)i;
        }
    }
}

__global__ void k_zero_u32(unsigned *p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *p = 0u;
}

enum { WEAK_SENS = 0, WEAK_UPDATE = 1, WEAK_STORE = 2, WEAK_ISRA = 3 };
static constexpr int kWeakThreads = 512;  // threads per weak voxel (a power of two)

// One block per listed voxel (j, r, s): the exact window sum
//   acc = sum_{taps inside the image} h[j][r mod N][s mod N][u][v] * img[r+u-c0][s+v-c0]
// in float64 (img == nullptr stands for an all-ones image, i.e. A^T 1).
//   WEAK_SENS:   sens[vox] = acc
//   WEAK_UPDATE: dst[vox] = sens[vox] > 0 ? src[vox] * acc / sens[vox] : 0
//   WEAK_STORE:  dst[vox] = acc
//   WEAK_ISRA:   dst[vox] = acc > 0 ? src[vox] * aux[vox] / acc : 0
__global__ void k_weak_exact(const unsigned *__restrict__ list, const float *__restrict__ psf,
                             int N, int K, int H, int W, const float *__restrict__ img,
                             float *__restrict__ sens, const float *__restrict__ src,
                             const float *__restrict__ aux, float *__restrict__ dst, int mode,
                             const int *__restrict__ skip)
{
    if (skip && *skip)
        return;
    __shared__ double red[kWeakThreads];
    const unsigned vox = list[blockIdx.x];
    const size_t hw = (size_t)H * W;
    const int j = (int)(vox / hw);
    const int r = (int)((vox % hw) / W), s = (int)(vox % W);
    const int c0 = (K - 1) / 2;
    const int u0 = max(0, c0 - r), u1 = min(K, H - r + c0);
    const int v0 = max(0, c0 - s), v1 = min(K, W - s + c0);
    const int wu = max(0, u1 - u0), wv = max(0, v1 - v0);
    const float *hk = psf + (((size_t)j * N + r % N) * N + s % N) * (size_t)K * K;
    double acc = 0.0;
    const int total = wu * wv;
    if (total > 0) {
        // tap idx = uu * wv + vv, advanced by blockDim.x without dividing per
        // tap; 8 taps' loads are issued before their products (clamped
        // addresses, taps past the window cleared by a mask)
        const int dq = blockDim.x / wv, dr = blockDim.x % wv;
        int uu = threadIdx.x / wv, vv = threadIdx.x % wv;
        for (int base = threadIdx.x; base < total; base += 8 * blockDim.x) {
            float hv[8], iv[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool ok = base + b * (int)blockDim.x < total;
                const int u = u0 + min(uu, wu - 1), v = v0 + vv;
                hv[b] = keep_if(hk[(size_t)u * K + v], ok);
                iv[b] = keep_if(img ? img[(size_t)(r + u - c0) * W + (s + v - c0)] : 1.0f, ok);
                uu += dq;
                vv += dr;
                if (vv >= wv) {
                    vv -= wv;
                    ++uu;
                }
            }
#pragma unroll
            for (int b = 0; b < 8; ++b)
                acc = fma((double)hv[b], (double)iv[b], acc);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (mode == WEAK_SENS) {
            sens[vox] = (float)red[0];
        } else if (mode == WEAK_UPDATE) {
            const float c = sens[vox];
            dst[vox] = c > 0.f ? (float)((double)src[vox] * red[0] / (double)c) : 0.f;
        } else if (mode == WEAK_STORE) {
            dst[vox] = (float)red[0];
        } else {
            dst[vox] = red[0] > 0.0 ? (float)((double)src[vox] * (double)aux[vox] / red[0]) : 0.f;
        }
    }
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
static constexpr int kDotBlocks = 512;

// Raise *flag when any of the n values is negative or not finite (an image RL
// cannot take: the ratio y / A x and the multiplicative update assume y >= 0).
__global__ void k_check_image(const float *__restrict__ a, size_t n, unsigned *__restrict__ flag)
{
    bool bad = false;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float v = a[i];
        bad |= !(v >= 0.f) || !(v <= 3.402823466e38f);
    }
    if (bad)
        atomicOr(flag, 1u);
}

// Scale each kernel of a PSF set to unit sum: one block per (j, a, b) kernel of
// n taps, the sum in float64, each tap divided in float64 and rounded once; a
// kernel whose sum is not positive is left unchanged.
__global__ void k_normalize_psf(float *__restrict__ psf, size_t n)
{
    __shared__ double red[256];
    float *h = psf + blockIdx.x * n;
    double a = 0.0;
    for (size_t i = threadIdx.x; i < n; i += blockDim.x)
        a += (double)h[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    const double s = red[0];
    if (!(s > 0.0))
        return;
    for (size_t i = threadIdx.x; i < n; i += blockDim.x)
        h[i] = (float)((double)h[i] / s);
}

// Device state of one frame's Richardson-Lucy run: the measured image, the
// ratio image, the iterates, A^T 1 with its weakly observed voxels, and the
// metric / stop state.  The plan holds one for lfrl_deconvolve; every job
// holds its own.  All device buffers are carved from one allocation.
struct Frame {
    int h = 0, w = 0;
    const float *y = nullptr;          // measured image [h][w]
    float *y_own = nullptr;            // the job's copy of it (jobs only)
    float *rho = nullptr;              // y / A x; the ones image while A^T 1 is formed
    float *V[2] = {nullptr, nullptr};  // x^{k-1} and x^k (ping-pong)
    float *VB = nullptr;               // best iterate under a metric stop mode
    float *sens = nullptr;             // A^T 1 [Nz][h][w]
    float *D = nullptr;                // A^T y [Nz][h][w] (ISRA numerator)
    unsigned *weak = nullptr;          // weakly observed voxels
    unsigned *counters = nullptr;      // [0] weak count, [1] bad-input flag
    unsigned *counters_host = nullptr; // pinned copy
    float *cmax = nullptr;             // [kDotBlocks + 1] max partials, max at [kDotBlocks]
    unsigned weak_cap = 0, nweak = 0;
    float *mip = nullptr;
    double *tabH = nullptr, *tabW = nullptr, *T1 = nullptr, *n2p = nullptr, *Fabs = nullptr;
    double *metric_out = nullptr, *trace = nullptr, *flux = nullptr, *dotp = nullptr;
    StopState *state = nullptr;
    StopState *state_host = nullptr;   // pinned, two slots (early-stop runs alternate them)
    int tab_h = -1, tab_nv = -1, tab_w = -1, tab_nu = -1;
    void *block = nullptr;             // the device allocation (owned by the job or plan)
    size_t block_bytes = 0;
    // run state
    lfrl_rl_opts opts{};
    bool want_flux = false;
    int iters = 0;
    bool done = false, stopped = false;
};

struct lfrl_plan_s {
    int device = 0;
    Geo g{};
    int max_h = 0, max_w = 0;
    int frame_tiles = 0;  // tiles of a max_h x max_w frame
    int max_tiles = 0;    // tiles one batched launch covers
    int split_k = 1;
    size_t resident = 0, workspace = 0;
    float2 *Gf = nullptr, *Gb = nullptr, *tw = nullptr;  // natural spectra (plan build only)
    float4 *Ff = nullptr, *Fb = nullptr;                 // FP32 spectra in fragment order
    float2 *Hx = nullptr;  // FP32: row xc of the adjoint spectra, [k][KKb] (xc >= 0)
    float2 *Gx = nullptr;  // FP32: column xcol of the forward spectra, [k][KKs] (xcol >= 0)
    float2 *X = nullptr, *Yp = nullptr, *Rs = nullptr;
    float *psf = nullptr;  // resident copy of the PSF set (weak-voxel sums)
    Frame fr;              // frame state of lfrl_deconvolve (sized for max_h x max_w)
    int sens_h = -1, sens_w = -1;
    // A^T 1 and weak-voxel lists of recent image sizes, copied into new jobs
    struct SensEntry {
        int h = 0, w = 0;
        float *sens = nullptr;
        unsigned *weak = nullptr;
        unsigned nweak = 0;
        size_t bytes = 0;
        unsigned long long stamp = 0;
    };
    std::vector<SensEntry> sens_cache;
    size_t sens_cache_bytes = 0, sens_cache_limit = 0;
    unsigned long long sens_clock = 0;
    size_t lds_r2c_bytes = 0, lds_c2r_bytes = 0, lds_r2c_vol_bytes = 0;
    bool use_fft = false;  // tile DFTs by the register FFT kernels
    int fwd_cb = 3, fwd_u = 4, adj_cb = 4, adj_u = 4;  // contraction launch shapes
    bool split = false;                 // split precision: 16-bit spectra (FP16 or BF16)
    bool bf16 = false;                  // ... in BF16 (LFRL_SPLIT_BF16)
    int hfwd_cb = 3, hfwd_u = 1, hadj_cb = 4, hadj_u = 2;  // their contraction shapes
    cplx16<_Float16> *Hf = nullptr, *Hb = nullptr;  // 16-bit spectra in fragment order
    int *gexp = nullptr;                // per-frequency exponents of the FP16 spectra
    unsigned *xmax = nullptr, *rmax = nullptr;  // per-(frequency, tile) maxima of tile spectra
    unsigned *rowpart = nullptr;                // their per-block parts (k_rowmax_reduce)
    int thr_r2c = 256, thr_c2r = 256;
    int c2r_stage = 0;        // inverse transform stages its epilogue inputs in LDS
    double tune_ms = 0.0;     // measured projection pair at the chosen tile (autotuned plans)
    // lfrl_deconvolve runs replayed from a captured graph (fixed-length stop modes)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    struct GraphKey {
        int h, w, max_iters, stop, patience, init, flux, update, region, norm, window;
        double xs, ys, background;
        const float *img;
        const float *vol;
        bool operator==(const GraphKey &o) const
        {
            return h == o.h && w == o.w && max_iters == o.max_iters && stop == o.stop &&
                   patience == o.patience && init == o.init && flux == o.flux &&
                   update == o.update && region == o.region && norm == o.norm &&
                   window == o.window && xs == o.xs && ys == o.ys &&
                   background == o.background && img == o.img && vol == o.vol;
        }
    } graph_key{};
    int graph_hits = 0;
    // early-stop runs: graphs of kStopChunk iterations each, by first iteration
    struct ChunkGraph {
        int k0;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<ChunkGraph> chunk_graphs;
    GraphKey chunk_key{};
    hipEvent_t chunk_ev[2] = {nullptr, nullptr};
    int tune_candidates = 0;  // tile sides timed
    // profiling
    bool prof = false;
    std::vector<hipEvent_t> ev[2];
    size_t ev_used[2] = {0, 0};
};

static int validate_desc(const lfrl_plan_desc *d)
{
    if (!d)
        return set_error(LFRL_ERR_ARG, "desc is NULL");
    if (d->nnum < 1 || d->nz < 1 || d->ksize < 1)
        return set_error(LFRL_ERR_ARG, "nnum, nz and ksize must be >= 1");
    if ((d->ksize & 1) == 0)
        return set_error(LFRL_ERR_ARG, "ksize must be odd (got %d)", d->ksize);
    if ((long long)d->nnum * d->nnum > kMaxNN)
        return set_error(LFRL_ERR_UNSUPPORTED, "nnum^2 must be <= %d", kMaxNN);
    if (d->max_h < d->nnum || d->max_w < d->nnum || d->max_h % d->nnum || d->max_w % d->nnum)
        return set_error(LFRL_ERR_ARG, "max_h/max_w must be positive multiples of nnum");
    if (d->precision != LFRL_FP32 && d->precision != LFRL_SPLIT_FP16 &&
        d->precision != LFRL_SPLIT_BF16)
        return set_error(LFRL_ERR_UNSUPPORTED, "precision %d not supported", d->precision);
    if (d->flags & ~(uint32_t)(LFRL_PLAN_AUTOTUNE | LFRL_NORMALIZE_PSF))
        return set_error(LFRL_ERR_ARG, "unknown plan flags 0x%x", d->flags);
    if (d->tile_q < 0 || d->tile_q > kMaxQ)
        return set_error(LFRL_ERR_ARG, "tile_q must be in [0, %d]", kMaxQ);
    if (d->max_batch < 0 || d->max_batch > kMaxBatchJobs)
        return set_error(LFRL_ERR_ARG, "max_batch must be in [0, %d]", kMaxBatchJobs);
    return LFRL_OK;
}

// Model of one iteration's time for tile side Q (bytes at a sustained HBM rate,
// flops at a sustained FP32 rate, the contraction overlapping its two bounds).
static bool fft_supported(int Q);

static double model_time(const Geo &g, const Tiles &t)
{
    const double nfu = unique_freqs(g.Q);   // frequencies the contractions visit
    const double spec = nfu * g.NN * g.KK * 8.0;
    const double inter = (double)g.nf * t.nt * (g.KK + g.NN) * 8.0;
    const double cflops = 8.0 * nfu * (double)g.NN * g.KK * t.nt;
    const double contract = 2.0 * std::max((spec + 2.0 * inter) / 5.0e12, cflops / 90.0e12);
    // tile transforms: both directions, volume side and image side
    const double tiles = (double)(g.KK + g.NN) * t.nt * 2.0;
    const double per_tile = fft_supported(g.Q)
                                ? 10.0 * g.Q * g.Q * std::log2((double)g.Q) / 40.0e12
                                : 12.0 * g.Q * g.Q * g.QH / 60.0e12;
    return contract + tiles * per_tile;
}

static size_t lds_limit()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
        return (size_t)v;
    return 160 * 1024;
}

// Tile sides a plan may use, ranked by the model (best first).  An explicit
// tile_q is the only candidate.
static int rank_q(const lfrl_plan_desc *d, size_t lds_max, std::vector<int> *out)
{
    Geo g;
    geo_init(g, d->nnum, d->nz, d->ksize, 1);
    const int R = g.R;
    out->clear();
    if (d->tile_q > 0) {
        if (d->tile_q < R)
            return set_error(LFRL_ERR_ARG, "tile_q %d smaller than the polyphase taps %d",
                             d->tile_q, R);
        Geo gq;
        geo_init(gq, d->nnum, d->nz, d->ksize, d->tile_q);
        if (lds_r2c(gq) > lds_max || lds_c2r(gq) > lds_max)
            return set_error(LFRL_ERR_UNSUPPORTED, "tile_q %d needs more LDS than available",
                             d->tile_q);
        if (d->precision != LFRL_FP32 && !fft_usable(gq, lds_max))
            return set_error(LFRL_ERR_UNSUPPORTED, "split FP16 needs an FFT tile size (tile_q %d)",
                             d->tile_q);
        out->push_back(d->tile_q);
        return LFRL_OK;
    }
    std::vector<std::pair<double, int>> ranked;
    for (int q = std::max(R, 2); q <= kMaxQ; ++q) {
        Geo gq;
        geo_init(gq, d->nnum, d->nz, d->ksize, q);
        if (lds_r2c(gq) > lds_max || lds_c2r(gq) > lds_max)
            continue;
        if (d->precision != LFRL_FP32 && !fft_usable(gq, lds_max))
            continue;  // the split path takes its row scales from the FFT tile kernels
        const Tiles t = tiles_for(gq, d->max_h, d->max_w);
        ranked.push_back({model_time(gq, t), q});
    }
    if (ranked.empty())
        return set_error(LFRL_ERR_UNSUPPORTED, "no DFT tile fits in %zu bytes of LDS", lds_max);
    // the model's choice: ascending q, a larger tile only when clearly faster
    size_t best = 0;
    for (size_t i = 1; i < ranked.size(); ++i)
        if (ranked[i].first < ranked[best].first * 0.999)
            best = i;
    out->push_back(ranked[best].second);
    ranked.erase(ranked.begin() + best);
    std::stable_sort(ranked.begin(), ranked.end(),
                     [](const std::pair<double, int> &x, const std::pair<double, int> &y) {
                         return x.first < y.first;
                     });
    for (auto &r : ranked)
        out->push_back(r.second);
    return LFRL_OK;
}

static int pick_q(const lfrl_plan_desc *d, size_t lds_max, int *q_out)
{
    std::vector<int> c;
    int rc = rank_q(d, lds_max, &c);
    if (rc)
        return rc;
    *q_out = c[0];
    return LFRL_OK;
}

static int pick_split(const Geo &g)
{
    int s = (2048 + g.nf - 1) / g.nf;
    // tuning override: LFRL_SPLIT_K (reduction chunks of the forward contraction)
    if (const char *e = getenv("LFRL_SPLIT_K"))
        if (atoi(e) > 0)
            s = atoi(e);
    s = std::max(1, std::min(s, (g.KK + 255) / 256));
    return s;
}

// Launch shapes of the two contractions: 16-column blocks per wave (CB) and
// prefetch depth in 4-deep reduction steps (U).  The forward spreads its
// NNp / 16 column blocks over at most 8 waves; the adjoint uses 4 waves.
static constexpr int kAdjWaves = 4;

// (U counts fragment pairs: two MFMA steps each)
static bool fwd_cb_ok(int cb) { return cb >= 2 && cb <= 5; }
static bool adj_cb_ok(int cb) { return cb == 2 || cb == 4; }
static bool u_ok(int u) { return u == 1 || u == 2 || u == 4; }

static void default_shapes(const Geo &g, int *fcb, int *fu, int *acb, int *au)
{
    // measured at Nnum 15 (14 matrix-core column blocks): 4 blocks per wave, 4 waves
    const int ncb = g.NNm / 16;
    int cb = std::max(2, std::min(5, (ncb + 3) / 4));
    while (cb < 5 && (ncb + cb - 1) / cb > 8)
        ++cb;
    *fcb = cb;
    *fu = 1;
    *acb = 4;
    *au = 1;
    // tuning override: LFRL_CONTRACT_SHAPE="fwd_cb,fwd_u,adj_cb,adj_u"
    const char *env = getenv("LFRL_CONTRACT_SHAPE");
    int a = 0, b = 0, c = 0, d = 0;
    if (env && sscanf(env, "%d,%d,%d,%d", &a, &b, &c, &d) == 4 && fwd_cb_ok(a) &&
        (ncb + a - 1) / a <= 8 && u_ok(b) && !(a >= 4 && b == 4) && adj_cb_ok(c) && u_ok(d)) {
        *fcb = a;
        *fu = b;
        *acb = c;
        *au = d;
    }
    // the forward stages its 64 * U A values per group with one per thread:
    // a block (one wave per CB column blocks) needs at least U waves
    const int fwaves = (ncb + *fcb - 1) / *fcb;
    while (*fu > fwaves)
        *fu /= 2;
}

static unsigned weak_cap_for(size_t nvox)
{
    size_t cap = std::min<size_t>(nvox, (size_t)1 << 20);
    // LFRL_WEAK_CAP lowers the list length (both its allocation and the
    // selection limit), so small frames can exercise the overflow refusal
    if (const char *e = getenv("LFRL_WEAK_CAP")) {
        const long v = atol(e);
        if (v > 0)
            cap = std::min<size_t>(cap, (size_t)v);
    }
    return (unsigned)std::max<size_t>(cap, 1);
}

// Device buffers of one Frame, in the order they are carved from its block.
enum {
    FB_Y, FB_RHO, FB_V0, FB_V1, FB_VB, FB_SENS, FB_D, FB_WEAK, FB_COUNTERS, FB_CMAX, FB_MIP, FB_TABH,
    FB_TABW, FB_T1, FB_N2P, FB_FABS, FB_MOUT, FB_TRACE, FB_FLUX, FB_DOTP, FB_STATE, FB_COUNT
};

// Byte offsets (256-byte aligned) of a Frame's buffers for an h x w image;
// returns the block size.  own_y: the frame keeps its own copy of the image.
// The metric buffers hold the whole coefficient matrix (LFRL_REGION_WHOLE).
static size_t frame_layout(const Geo &g, int h, int w, bool own_y, size_t off[FB_COUNT])
{
    const size_t hw = (size_t)h * w, nvox = (size_t)g.Nz * hw;
    const size_t legs_h = std::min(h, kMaxMetricLegs);
    size_t bytes[FB_COUNT];
    bytes[FB_Y] = own_y ? hw * sizeof(float) : 0;
    bytes[FB_RHO] = hw * sizeof(float);
    bytes[FB_V0] = bytes[FB_V1] = bytes[FB_VB] = bytes[FB_SENS] = bytes[FB_D] =
        nvox * sizeof(float);
    bytes[FB_WEAK] = (size_t)weak_cap_for(nvox) * sizeof(unsigned);
    bytes[FB_COUNTERS] = 2 * sizeof(unsigned);
    bytes[FB_CMAX] = (kDotBlocks + 1) * sizeof(float);
    bytes[FB_MIP] = hw * sizeof(float);
    bytes[FB_TABH] = (size_t)h * h * sizeof(double);
    bytes[FB_TABW] = (size_t)w * w * sizeof(double);
    bytes[FB_T1] = std::max((size_t)kMetricChunks * legs_h * w, hw) * sizeof(double);
    bytes[FB_N2P] = ((hw + 255) / 256 + 1) * sizeof(double);  // + the spectral norm
    bytes[FB_FABS] = hw * sizeof(double);
    bytes[FB_MOUT] = sizeof(double);
    bytes[FB_TRACE] = bytes[FB_FLUX] = (size_t)kMaxTrace * sizeof(double);
    bytes[FB_DOTP] = (size_t)kDotBlocks * sizeof(double);
    bytes[FB_STATE] = sizeof(StopState);
    size_t total = 0;
    for (int i = 0; i < FB_COUNT; ++i) {
        off[i] = total;
        total += (bytes[i] + 255) / 256 * 256;
    }
    return total;
}

static void frame_bind(Frame &f, const Geo &g, int h, int w, void *block, const size_t off[FB_COUNT],
                       bool own_y)
{
    char *b = (char *)block;
    f.h = h;
    f.w = w;
    f.y_own = own_y ? (float *)(b + off[FB_Y]) : nullptr;
    f.rho = (float *)(b + off[FB_RHO]);
    f.V[0] = (float *)(b + off[FB_V0]);
    f.V[1] = (float *)(b + off[FB_V1]);
    f.VB = (float *)(b + off[FB_VB]);
    f.sens = (float *)(b + off[FB_SENS]);
    f.D = (float *)(b + off[FB_D]);
    f.weak = (unsigned *)(b + off[FB_WEAK]);
    f.counters = (unsigned *)(b + off[FB_COUNTERS]);
    f.cmax = (float *)(b + off[FB_CMAX]);
    f.mip = (float *)(b + off[FB_MIP]);
    f.tabH = (double *)(b + off[FB_TABH]);
    f.tabW = (double *)(b + off[FB_TABW]);
    f.T1 = (double *)(b + off[FB_T1]);
    f.n2p = (double *)(b + off[FB_N2P]);
    f.Fabs = (double *)(b + off[FB_FABS]);
    f.metric_out = (double *)(b + off[FB_MOUT]);
    f.trace = (double *)(b + off[FB_TRACE]);
    f.flux = (double *)(b + off[FB_FLUX]);
    f.dotp = (double *)(b + off[FB_DOTP]);
    f.state = (StopState *)(b + off[FB_STATE]);
    f.weak_cap = weak_cap_for((size_t)g.Nz * h * w);
    f.nweak = 0;
    f.tab_h = f.tab_nv = f.tab_w = f.tab_nu = -1;
}

struct Sizes {
    size_t Gf, Gb, tw, psf, X, Yp, Rs, frame;  // Gf, Gb: natural layouts, plan build only
    size_t Ff = 0, Fb = 0;                      // FP32 fragment-ordered spectra
    size_t Hx = 0;                              // FP32: spectra row of the lone adjoint index
    size_t Gx = 0;                              // FP32: spectra column of the lone output column
    size_t Hf = 0, Hb = 0, gexp = 0, rowmax = 0, rowpart = 0;  // split FP16 only
    bool split = false;
    size_t resident() const { return (split ? Hf + Hb + gexp : Ff + Fb) + Hx + Gx + tw + psf; }
    size_t workspace() const { return X + Yp + Rs + 2 * rowmax + rowpart + frame; }
};

static Sizes sizes_for(const Geo &g, int max_h, int max_w, int max_batch, int split, bool f16)
{
    const int nt = tiles_for(g, max_h, max_w).nt * std::max(1, max_batch);
    Sizes s;
    s.Gf = (size_t)g.nf * g.NNp * g.KK * sizeof(float2);
    s.Gb = (size_t)g.nf * g.NN * g.KK * sizeof(float2);
    s.Ff = (size_t)g.nf * g.KKs * g.NNm * sizeof(float2);
    s.Gx = g.xcol >= 0 ? (size_t)g.nf * g.KKs * sizeof(float2) : 0;
    s.Fb = (size_t)g.nf * g.NCm * g.KKb * sizeof(float2);
    s.Hx = g.xc >= 0 ? (size_t)g.nf * g.KKb * sizeof(float2) : 0;
    s.tw = (size_t)g.Q * sizeof(float2);
    s.X = (size_t)g.nf * nt * g.KKs * sizeof(float2);
    s.Yp = (size_t)split * g.nf * nt * g.NN * sizeof(float2);
    s.Rs = (size_t)g.nf * nt * g.NN * sizeof(float2);
    s.psf = (size_t)g.Nz * g.NN * g.K * g.K * sizeof(float);
    size_t off[FB_COUNT];
    s.frame = frame_layout(g, max_h, max_w, false, off);
    if (f16) {
        s.split = true;
        s.Hf = (size_t)g.nf * g.KKs * g.NNm * sizeof(cplx16<_Float16>);
        s.Hb = (size_t)g.nf * g.NNm * ((g.KK + 15) / 16 * 16) * sizeof(cplx16<_Float16>);
        s.gexp = (size_t)g.nf * sizeof(int);
        s.rowmax = (size_t)g.nf * nt * sizeof(unsigned);
        // per-block maxima of the volume transform (the image's fit in them)
        s.rowpart = (size_t)g.Nz * g.N * nt * g.nf * sizeof(unsigned);
    }
    return s;
}

// Check that [ptr, ptr + bytes) lies inside one device allocation, so a host
// pointer or a short buffer is reported as an argument error instead of
// faulting the GPU.
static constexpr size_t kTuneCandidatesFp = 4;  // tile sides an autotuned plan times

static int check_buf(const void *ptr, size_t bytes, const char *name)
{
    if (!ptr)
        return set_error(LFRL_ERR_ARG, "%s is NULL", name);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    hipError_t e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(LFRL_ERR_ARG, "%s is not a device allocation", name);
    }
    const char *b = (const char *)base, *q = (const char *)ptr;
    if (q < b || (size_t)(q - b) + bytes > size)
        return set_error(LFRL_ERR_ARG, "%s: %zu bytes do not fit in its allocation", name, bytes);
    return LFRL_OK;
}

extern "C" int lfrl_plan_footprint(const lfrl_plan_desc *desc, size_t *resident_bytes,
                                   size_t *workspace_bytes)
{
    int rc = validate_desc(desc);
    if (rc)
        return rc;
    std::vector<int> cands;
    rc = rank_q(desc, 160 * 1024, &cands);
    if (rc)
        return rc;
    // an autotuned plan may take any of the timed candidates: report the largest
    const size_t n = (desc->flags & LFRL_PLAN_AUTOTUNE)
                         ? std::min<size_t>(cands.size(), kTuneCandidatesFp)
                         : 1;
    size_t res = 0, ws = 0;
    for (size_t i = 0; i < n; ++i) {
        Geo g;
        geo_init(g, desc->nnum, desc->nz, desc->ksize, cands[i]);
        const Sizes s = sizes_for(g, desc->max_h, desc->max_w, desc->max_batch, pick_split(g),
                                  desc->precision != LFRL_FP32);
        res = std::max(res, s.resident());
        ws = std::max(ws, s.workspace());
    }
    if (resident_bytes)
        *resident_bytes = res;
    if (workspace_bytes)
        *workspace_bytes = ws;
    return LFRL_OK;
}

static void free_frame(Frame &f)
{
    if (f.block)
        (void)hipFree(f.block);
    if (f.state_host)
        (void)hipHostFree(f.state_host);
    if (f.counters_host)
        (void)hipHostFree(f.counters_host);
    f.block = nullptr;
    f.state_host = nullptr;
    f.counters_host = nullptr;
}

static void free_plan(lfrl_plan_s *p)
{
    if (!p)
        return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    void *bufs[] = {p->Gf, p->Gb, p->Ff, p->Fb, p->Hx, p->Gx, p->tw, p->X, p->Yp, p->Rs, p->psf,
                    p->Hf, p->Hb, p->gexp, p->xmax, p->rmax, p->rowpart};
    for (void *b : bufs)
        if (b)
            (void)hipFree(b);
    free_frame(p->fr);
    for (auto &e : p->sens_cache) {
        (void)hipFree(e.sens);
        (void)hipFree(e.weak);
    }
    for (auto &c : p->chunk_graphs) {
        (void)hipGraphExecDestroy(c.exec);
        (void)hipGraphDestroy(c.graph);
    }
    p->chunk_graphs.clear();
    for (hipEvent_t e : p->chunk_ev)
        if (e)
            (void)hipEventDestroy(e);
    if (p->graph_exec)
        (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    if (p->cap_stream)
        (void)hipStreamDestroy(p->cap_stream);
    for (auto &v : p->ev)
        for (hipEvent_t e : v)
            (void)hipEventDestroy(e);
    (void)hipSetDevice(cur);
    delete p;
}

template <typename T>
static int dalloc(T **ptr, size_t bytes)
{
    hipError_t e = hipMalloc((void **)ptr, bytes ? bytes : 16);
    if (e != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return set_error(LFRL_ERR_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    return LFRL_OK;
}

// Allocate and bind a Frame's device block and pinned host words.
// Device blocks of jobs come from a per-device pool: a released job's block
// and pinned words are kept and handed to a later job of the same size class,
// so the serving loop does not call hipMalloc / hipFree (which synchronises
// the device) per request.  Sizes are rounded up to classes about 6% apart;
// lfrl_job_footprint reports the rounded size.
static size_t job_size_class(size_t bytes)
{
    size_t c = 1 << 20;
    while (c < bytes && c * 2 > c)
        c *= 2;
    if (c <= (1 << 20))
        return c;
    const size_t step = c / 32;  // 16 classes per octave
    return (bytes + step - 1) / step * step;
}

struct JobSlot {
    void *block = nullptr;
    size_t bytes = 0;
    StopState *state_host = nullptr;
    unsigned *counters_host = nullptr;
    hipEvent_t used = nullptr;  // recorded after the last work queued on the job
};
static std::mutex g_slot_mu;
static std::vector<std::vector<JobSlot>> g_slots;  // [device] free slots

static void slot_release_all(int dev)
{
    std::vector<JobSlot> v;
    {
        std::lock_guard<std::mutex> lk(g_slot_mu);
        if ((int)g_slots.size() > dev)
            v.swap(g_slots[dev]);
    }
    for (JobSlot &s : v) {
        (void)hipFree(s.block);
        (void)hipHostFree(s.state_host);
        (void)hipHostFree(s.counters_host);
        (void)hipEventDestroy(s.used);
    }
}

// A slot of exactly `bytes` (a size class) from the pool, else a new one.
static int slot_get(int dev, size_t bytes, JobSlot *out)
{
    {
        std::lock_guard<std::mutex> lk(g_slot_mu);
        if ((int)g_slots.size() > dev) {
            auto &v = g_slots[dev];
            for (size_t i = 0; i < v.size(); ++i)
                if (v[i].bytes == bytes) {
                    *out = v[i];
                    v[i] = v.back();
                    v.pop_back();
                    return LFRL_OK;
                }
        }
    }
    JobSlot s;
    s.bytes = bytes;
    hipError_t e = hipMalloc(&s.block, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        slot_release_all(dev);  // cached blocks of other classes may be in the way
        e = hipMalloc(&s.block, bytes);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(LFRL_ERR_NOMEM, "hipMalloc(%zu) for a job failed: %s", bytes,
                         hipGetErrorString(e));
    }
    e = hipHostMalloc((void **)&s.state_host, 2 * sizeof(StopState), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&s.counters_host, 2 * sizeof(unsigned), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&s.used, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(s.block);
        if (s.state_host)
            (void)hipHostFree(s.state_host);
        if (s.counters_host)
            (void)hipHostFree(s.counters_host);
        return set_error(LFRL_ERR_NOMEM, "hipHostMalloc failed: %s", hipGetErrorString(e));
    }
    *out = s;
    return LFRL_OK;
}

static void slot_put(int dev, const JobSlot &s)
{
    std::lock_guard<std::mutex> lk(g_slot_mu);
    if ((int)g_slots.size() <= dev)
        g_slots.resize(dev + 1);
    g_slots[dev].push_back(s);
}

static int frame_alloc(Frame &f, const Geo &g, int h, int w, bool own_y)
{
    size_t off[FB_COUNT];
    const size_t bytes = frame_layout(g, h, w, own_y, off);
    int rc = dalloc((char **)&f.block, bytes);
    if (rc)
        return rc;
    f.block_bytes = bytes;
    frame_bind(f, g, h, w, f.block, off, own_y);
    hipError_t e = hipHostMalloc((void **)&f.state_host, 2 * sizeof(StopState), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&f.counters_host, 2 * sizeof(unsigned), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_frame(f);
        return set_error(LFRL_ERR_NOMEM, "hipHostMalloc failed: %s", hipGetErrorString(e));
    }
    return LFRL_OK;
}

#define TRY(expr)              \
    do {                       \
        int rc_ = (expr);      \
        if (rc_ != LFRL_OK) {  \
            free_plan(p);      \
            return rc_;        \
        }                      \
    } while (0)

static void set_lds_attrs(size_t lds)
{
    raise_lds_attr((const void *)k_psf_r2c, lds);
    raise_lds_attr((const void *)k_vol_r2c, lds);
    raise_lds_attr((const void *)k_c2r, lds);
}

// Allocate a plan for tile side q and build its spectra from `psf`.  With
// psf == nullptr the plan is for timing only: its spectra are zero, it has no
// PSF copy and no frame state (lfrl_deconvolve cannot run on it).
static int plan_build(lfrl_plan_s **out, const lfrl_plan_desc *desc, int q, const float *psf,
                      hipStream_t st)
{
    *out = nullptr;
    const bool timing = psf == nullptr;
    const size_t lmax = lds_limit();
    lfrl_plan_s *p = new lfrl_plan_s();
    {
        hipError_t e0 = hipGetDevice(&p->device);
        if (e0 != hipSuccess) {
            delete p;
            return set_error(LFRL_ERR_DEVICE, "hipGetDevice failed: %s", hipGetErrorString(e0));
        }
    }
    geo_init(p->g, desc->nnum, desc->nz, desc->ksize, q);
    const Geo &g = p->g;
    p->max_h = desc->max_h;
    p->max_w = desc->max_w;
    p->frame_tiles = tiles_for(g, desc->max_h, desc->max_w).nt;
    p->max_tiles = p->frame_tiles * std::max(1, (int)desc->max_batch);
    // the inverse tile DFTs address one frequency row of a launch's tile
    // spectra with 32-bit byte offsets
    if ((size_t)g.QH * g.KKs * p->max_tiles * sizeof(float2) >= ((size_t)1 << 32)) {
        free_plan(p);
        return set_error(LFRL_ERR_UNSUPPORTED, "tile spectra of %d tiles too large", p->max_tiles);
    }
    p->split_k = pick_split(g);
    p->split = desc->precision != LFRL_FP32;
    p->bf16 = desc->precision == LFRL_SPLIT_BF16;
    const Sizes s = sizes_for(g, p->max_h, p->max_w, desc->max_batch, p->split_k, p->split);
    p->resident = s.resident();
    p->workspace = s.workspace();
    p->use_fft = fft_usable(g, lmax);
    default_shapes(g, &p->fwd_cb, &p->fwd_u, &p->adj_cb, &p->adj_u);
    {
        const char *env = getenv("LFRL_SENS_CACHE_MB");
        const long mb = env ? atol(env) : 2048;
        p->sens_cache_limit = (size_t)std::max(0L, mb) << 20;
    }
    {
        // split FP16 shapes; tuning override LFRL_CONTRACT_SHAPE_F16="fcb,fu,acb,au"
        const int ncb = g.NNm / 16;
        p->hfwd_cb = ncb > 8 ? 2 : 1;
        if ((ncb + p->hfwd_cb - 1) / p->hfwd_cb > 8)
            p->hfwd_cb = 3;
        const char *env = getenv("LFRL_CONTRACT_SHAPE_F16");
        int a = 0, b = 0, c = 0, d = 0;
        // (only shapes whose registers fit without spilling)
        if (env && sscanf(env, "%d,%d,%d,%d", &a, &b, &c, &d) == 4 &&
            ((a == 1 || a == 2) ? (b == 1 || b == 2) : (a == 3 && b == 1)) &&
            (ncb + a - 1) / a <= 8 && (c == 2 || c == 4) && (d == 2 || d == 4)) {
            p->hfwd_cb = a;
            p->hfwd_u = b;
            p->hadj_cb = c;
            p->hadj_u = d;
        }
    }
    if (p->use_fft) {
        p->lds_r2c_bytes = lds_r2c_fft(g);
        p->lds_r2c_vol_bytes = lds_r2c_fft_planes(g);
        p->c2r_stage = c2r_stage_fits(g, lmax);
        if (const char *e = getenv("LFRL_C2R_STAGE"))  // tuning override: 0 or 1
            p->c2r_stage = atoi(e) != 0 && c2r_stage_bytes(g) + lds_c2r_fft(g) <= lmax;
        p->lds_c2r_bytes = lds_c2r_fft(g) + (p->c2r_stage ? c2r_stage_bytes(g) : 0);
        p->thr_r2c = threads_r2c_fft(g);
        p->thr_c2r = threads_c2r_fft(g);
    } else {
        p->lds_r2c_bytes = p->lds_r2c_vol_bytes = lds_r2c(g);
        p->lds_c2r_bytes = lds_c2r(g);
    }
    if (!timing) {
        TRY(dalloc(&p->Gf, s.Gf));
        TRY(dalloc(&p->Gb, s.Gb));
    }
    if (!p->split) {
        TRY(dalloc(&p->Ff, s.Ff));
        TRY(dalloc(&p->Fb, s.Fb));
    }
    if (s.Hx)
        TRY(dalloc(&p->Hx, s.Hx));
    if (s.Gx)
        TRY(dalloc(&p->Gx, s.Gx));
    TRY(dalloc(&p->tw, s.tw));
    TRY(dalloc(&p->X, s.X));
    TRY(dalloc(&p->Yp, s.Yp));
    TRY(dalloc(&p->Rs, s.Rs));
    if (!timing) {
        TRY(dalloc(&p->psf, s.psf));
        TRY(frame_alloc(p->fr, g, p->max_h, p->max_w, false));
    }
    if (p->split) {
        TRY(dalloc(&p->Hf, s.Hf));
        TRY(dalloc(&p->Hb, s.Hb));
        TRY(dalloc(&p->gexp, s.gexp));
        TRY(dalloc(&p->xmax, s.rowmax));
        TRY(dalloc(&p->rmax, s.rowmax));
        TRY(dalloc(&p->rowpart, s.rowpart));
    }
    // twiddles exp(2 pi i m / Q), computed in double, rounded once
    std::vector<float2> tw(g.Q);
    for (int m = 0; m < g.Q; ++m) {
        const double th = 2.0 * M_PI * (double)m / (double)g.Q;
        tw[m] = make_float2((float)std::cos(th), (float)std::sin(th));
    }
    const size_t lds_fft = std::max({p->lds_r2c_bytes, p->lds_r2c_vol_bytes, p->lds_c2r_bytes});
    set_lds_attrs(lds_fft);
    if (p->use_fft)
        set_fft_lds_attrs(g.Q, lds_fft);
    hipError_t e = hipMemcpyAsync(p->tw, tw.data(), g.Q * sizeof(float2), hipMemcpyHostToDevice, st);
    if (timing) {
        // zero spectra: the projections' cost does not depend on the values
        if (e == hipSuccess)
            e = p->split ? hipMemsetAsync(p->Hf, 0, s.Hf, st) : hipMemsetAsync(p->Ff, 0, s.Ff, st);
        if (e == hipSuccess)
            e = p->split ? hipMemsetAsync(p->Hb, 0, s.Hb, st) : hipMemsetAsync(p->Fb, 0, s.Fb, st);
        if (e == hipSuccess && s.Hx)
            e = hipMemsetAsync(p->Hx, 0, s.Hx, st);
        if (e == hipSuccess && s.Gx)
            e = hipMemsetAsync(p->Gx, 0, s.Gx, st);
        if (e == hipSuccess && p->split)
            e = hipMemsetAsync(p->gexp, 0, s.gexp, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            free_plan(p);
            return set_error(LFRL_ERR_DEVICE, "plan build failed: %s", hipGetErrorString(e));
        }
        *out = p;
        return LFRL_OK;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->psf, psf, s.psf, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && (desc->flags & LFRL_NORMALIZE_PSF)) {
        hipLaunchKernelGGL(k_normalize_psf, dim3(g.Nz * g.NN), dim3(256), 0, st, p->psf,
                           (size_t)g.K * g.K);
        e = hipGetLastError();
    }
    // everything below is built from the plan's own copy
    psf = p->psf;
    if (e == hipSuccess && g.NNp != g.NN)
        e = hipMemsetAsync(p->Gf, 0, s.Gf, st);  // zero the row padding
    if (e == hipSuccess) {
        dim3 grid(g.N, g.NN, g.Nz);
        if (p->use_fft)
            launch_r2c_fft(g.Q, grid, p->thr_r2c, p->lds_r2c_bytes, st, SRC_PSF, TileBatch{}, psf,
                           g.N, g.T, g.hD, 0, g.NNp, g.K, g.c0, g.KK, p->Gf, p->tw);
        else
            hipLaunchKernelGGL(k_psf_r2c, grid, dim3(256), p->lds_r2c_bytes, st, psf, g.N, g.K,
                               g.c0, g.hD, g.Q, g.QH, g.KK, g.NNp, p->Gf, p->tw);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        dim3 grid((g.NN + 31) / 32, (g.KK + 31) / 32, g.nf);
        hipLaunchKernelGGL(k_transpose_spec, grid, dim3(32, 8), 0, st, p->Gf, p->Gb, g.KK, g.NN,
                           g.NNp);
        e = hipGetLastError();
    }
    if (e == hipSuccess && p->split) {
        // 16-bit fragments with per-frequency power-of-two scales
        hipLaunchKernelGGL(k_spec_exp, dim3(g.nf), dim3(256), 0, st, (const float2 *)p->Gf,
                           (size_t)g.KK * g.NNp, p->gexp);
        const size_t nhf = s.Hf / sizeof(cplx16<_Float16>), nhb = s.Hb / sizeof(cplx16<_Float16>);
        if (p->bf16) {
            hipLaunchKernelGGL(k_pack_fwd_split<PrecBF16>, dim3(8192), dim3(256), 0, st,
                               (const float2 *)p->Gf, g.KK, g.NNp, g.NNm / 16, g.KKs / 32,
                               (const int *)p->gexp, (cplx16<__bf16> *)p->Hf, nhf);
            hipLaunchKernelGGL(k_pack_adj_split<PrecBF16>, dim3(8192), dim3(256), 0, st,
                               (const float2 *)p->Gb, g.NN, g.KK, g.NNm / 16, (g.KK + 15) / 16,
                               (const int *)p->gexp, (cplx16<__bf16> *)p->Hb, nhb);
        } else {
            hipLaunchKernelGGL(k_pack_fwd_split<PrecF16>, dim3(8192), dim3(256), 0, st,
                               (const float2 *)p->Gf, g.KK, g.NNp, g.NNm / 16, g.KKs / 32,
                               (const int *)p->gexp, p->Hf, nhf);
            hipLaunchKernelGGL(k_pack_adj_split<PrecF16>, dim3(8192), dim3(256), 0, st,
                               (const float2 *)p->Gb, g.NN, g.KK, g.NNm / 16, (g.KK + 15) / 16,
                               (const int *)p->gexp, p->Hb, nhb);
        }
        e = hipGetLastError();
    } else if (e == hipSuccess) {
        // FP32 fragments
        hipLaunchKernelGGL(k_pack_fwd_f32, dim3(8192), dim3(256), 0, st, (const float2 *)p->Gf,
                           g.KK, g.NNp, g.NNm / 16, g.KKs, p->Ff, s.Ff / sizeof(float4));
        hipLaunchKernelGGL(k_pack_adj_f32, dim3(8192), dim3(256), 0, st, (const float2 *)p->Gb,
                           g.NN, g.KK, g.NCm, g.KKb, p->adj_cb * kAdjWaves, p->Fb,
                           s.Fb / sizeof(float4));
        e = hipGetLastError();
    }
    // float32 row / column of the lone indices (both precisions)
    if (e == hipSuccess && s.Gx) {
        hipLaunchKernelGGL(k_spec_column, dim3(2048), dim3(256), 0, st, (const float2 *)p->Gf, g.KK,
                           g.NNp, g.KKs, g.xcol, p->Gx, (size_t)g.nf * g.KKs);
        e = hipGetLastError();
    }
    if (e == hipSuccess && s.Hx) {
        // Hx[k][kk] = Gb[k][xc][kk], zero past KK
        e = hipMemsetAsync(p->Hx, 0, s.Hx, st);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(p->Hx, (size_t)g.KKb * sizeof(float2),
                                 p->Gb + (size_t)g.xc * g.KK, (size_t)g.NN * g.KK * sizeof(float2),
                                 (size_t)g.KK * sizeof(float2), (size_t)g.nf,
                                 hipMemcpyDeviceToDevice, st);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
        // the natural-layout spectra were only the packers' input
        (void)hipFree(p->Gf);
        (void)hipFree(p->Gb);
        p->Gf = p->Gb = nullptr;
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);  // the tw staging vector goes out of scope
    if (e != hipSuccess) {
        free_plan(p);
        return set_error(LFRL_ERR_DEVICE, "plan build failed: %s", hipGetErrorString(e));
    }
    *out = p;
    return LFRL_OK;
}

#undef TRY

static constexpr int kTuneCandidates = (int)kTuneCandidatesFp;
static int autotune_q(const lfrl_plan_desc *desc, const std::vector<int> &cands, hipStream_t st,
                      int *q_out, double *ms_out, int *tried);

extern "C" int lfrl_plan(lfrl_plan_t *out, const lfrl_plan_desc *desc, const float *psf,
                         void *stream)
{
    if (!out)
        return set_error(LFRL_ERR_ARG, "out is NULL");
    *out = nullptr;
    int rc = validate_desc(desc);
    if (rc)
        return rc;
    if (!psf)
        return set_error(LFRL_ERR_ARG, "psf is NULL");
    hipStream_t st = (hipStream_t)stream;
    std::vector<int> cands;
    if ((rc = rank_q(desc, lds_limit(), &cands)))
        return rc;
    rc = check_buf(psf, (size_t)desc->nz * desc->nnum * desc->nnum * desc->ksize * desc->ksize *
                            sizeof(float), "psf");
    if (rc)
        return rc;
    int q = cands[0], tried = 0;
    double tune_ms = 0.0;
    if ((desc->flags & LFRL_PLAN_AUTOTUNE) && cands.size() > 1 &&
        (rc = autotune_q(desc, cands, st, &q, &tune_ms, &tried)))
        return rc;
    lfrl_plan_s *p = nullptr;
    if ((rc = plan_build(&p, desc, q, psf, st)))
        return rc;
    p->tune_ms = tune_ms;
    p->tune_candidates = tried;
    // the graph-capture stream and the early-stop events, made here so that
    // later calls create nothing
    hipError_t e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    for (hipEvent_t &ev : p->chunk_ev)
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        free_plan(p);
        return set_error(LFRL_ERR_DEVICE, "plan stream/events: %s", hipGetErrorString(e));
    }
    *out = p;
    return LFRL_OK;
}

extern "C" int lfrl_plan_destroy(lfrl_plan_t plan)
{
    free_plan(plan);
    return LFRL_OK;
}

extern "C" int lfrl_plan_get_info(lfrl_plan_t p, lfrl_plan_info_t *info)
{
    if (!p || !info)
        return set_error(LFRL_ERR_ARG, "NULL argument");
    info->tile_q = p->g.Q;
    info->tile_out = p->g.T;
    info->taps = p->g.R;
    info->nfreq = p->g.nf;
    info->nfreq_unique = unique_freqs(p->g.Q);
    info->max_tiles = p->max_tiles;
    info->split_k = p->split_k;
    info->resident_bytes = p->resident;
    info->workspace_bytes = p->workspace;
    info->tune_candidates = p->tune_candidates;
    info->tune_ms = p->tune_ms;
    return LFRL_OK;
}

// ---------------------------------------------------------------------------
// internal launches
// ---------------------------------------------------------------------------
struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        if (prev != dev)
            (void)hipSetDevice(dev);
    }
    ~DevGuard()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

static int check_hw(lfrl_plan_s *p, int h, int w)
{
    if (h < p->g.N || w < p->g.N || h % p->g.N || w % p->g.N)
        return set_error(LFRL_ERR_ARG, "h=%d, w=%d must be positive multiples of nnum=%d", h, w, p->g.N);
    if (h > p->max_h || w > p->max_w)
        return set_error(LFRL_ERR_ARG, "image %dx%d exceeds the plan maximum %dx%d", h, w,
                         p->max_h, p->max_w);
    return LFRL_OK;
}

static int prof_event(lfrl_plan_s *p, int which, hipStream_t st)
{
    auto &v = p->ev[which];
    size_t &used = p->ev_used[which];
    if (used == v.size()) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        v.push_back(e);
    }
    HIP_TRY(hipEventRecord(v[used++], st));
    return LFRL_OK;
}

#define LFRL_FWD_CASE(CBV, UV)                                                                   \
    if (p->fwd_cb == CBV && p->fwd_u == UV) {                                                    \
        hipLaunchKernelGGL((k_contract_fwd<CBV, UV>), grid, block, 0, st, (const float4 *)p->Ff, \
                           (const float2 *)p->X, p->Yp, g.NN, g.NNm, g.KK, g.KKs, nt, g.nf,     \
                           kchunk, skip, freq_map(g.Q),                                          \
                           (const float4 *)(p->Gx ? p->Gx : (float2 *)p->Ff), g.xcol);           \
        launched = true;                                                                         \
    }
#define LFRL_FWD_CASES(CBV) LFRL_FWD_CASE(CBV, 1) LFRL_FWD_CASE(CBV, 2) LFRL_FWD_CASE(CBV, 4)
#define LFRL_ADJ_CASE(CBV, UV)                                                                   \
    if (p->adj_cb == CBV && p->adj_u == UV) {                                                    \
        hipLaunchKernelGGL((k_contract_adj<CBV, UV>), grid, dim3(64 * kAdjWaves), lds, st,       \
                           (const float4 *)p->Fb, (const float2 *)p->Rs, p->X, g.NN, g.KK,      \
                           g.KKs, g.NCm, nt, ranges, skip, freq_map(g.Q), (const float2 *)p->Hx, \
                           g.xc, g.KKb, osk, ost);                                               \
        launched = true;                                                                         \
    }
#define LFRL_ADJ_CASES(CBV) LFRL_ADJ_CASE(CBV, 1) LFRL_ADJ_CASE(CBV, 2) LFRL_ADJ_CASE(CBV, 4)

static int contraction_split(const lfrl_plan_s *p, int *kchunk)
{
    const Geo &g = p->g;
    int kc = (g.KK + p->split_k - 1) / p->split_k;
    kc = (kc + 63) / 64 * 64;
    *kchunk = kc;
    return (g.KK + kc - 1) / kc;
}

// One frame of a batched tile launch: its size, the array the forward tile
// transform reads, and the inverse transform's destination and epilogue inputs.
struct FrameIO {
    int h, w;
    const float *src;
    float *dst;
    const float *aux0, *aux1;
    float bg = 0.f;  // background of EPI_STORE / EPI_RATIO
    int mode = -1;   // epilogue of this frame (-1: the launch's)
    const int *skip = nullptr;  // device flag: nonzero = the frame's work is skipped
};

// Concatenate the frames' tiles into one tile index space; returns the total.
static int make_batch(const Geo &g, const FrameIO *io, int n, int mode, TileBatch *b)
{
    int nt = 0;
    b->njobs = n;
    for (int i = 0; i < n; ++i) {
        const Tiles t = tiles_for(g, io[i].h, io[i].w);
        TileJob &j = b->job[i];
        j.src = io[i].src;
        j.dst = io[i].dst;
        j.aux0 = io[i].aux0;
        j.aux1 = io[i].aux1;
        j.bg = io[i].bg;
        j.mode = io[i].mode >= 0 ? io[i].mode : mode;
        j.skip = io[i].skip;
        j.H = io[i].h;
        j.W = io[i].w;
        j.tiles_x = t.tx;
        j.tile0 = nt;
        nt += t.nt;
    }
    return nt;
}

// Forward projection of n frames in one pass: vol [Nz][h][w] -> img [h][w]
// per frame, stored (mode STORE) or turned into the RL ratio y / (A x)
// (mode RATIO, y = aux0).  The frames' tiles share every launch; their total
// must not exceed the plan's tile capacity.
static int run_forward(lfrl_plan_s *p, const FrameIO *io, int n, int mode, hipStream_t st)
{
    const Geo &g = p->g;
    TileBatch batch;
    const int nt = make_batch(g, io, n, mode, &batch);
    if (nt > p->max_tiles)
        return set_error(LFRL_ERR_ARG, "batch of %d tiles exceeds the plan capacity %d", nt,
                         p->max_tiles);
    // a launch of one frame stops with it; frames of a batch share the launch
    const int *skip = n == 1 ? io[0].skip : nullptr;
    if (p->use_fft)
        launch_r2c_fft(g.Q, dim3(nt * g.Nz * g.N), p->thr_r2c, p->lds_r2c_vol_bytes, st, SRC_PLANES,
                       batch, nullptr, g.N, g.T, g.hD, nt, g.KKs, g.K, g.c0, g.KK, p->X, p->tw,
                       p->split ? p->rowpart : nullptr);
    else
        hipLaunchKernelGGL(k_vol_r2c, dim3(nt, g.Nz * g.N), dim3(256), p->lds_r2c_bytes, st, batch,
                           g.N, g.Q, g.QH, g.T, g.hD, nt, g.KKs, p->X, p->tw);
    LAUNCH_CHECK("k_vol_r2c");
    if (p->split) {
        hipLaunchKernelGGL(k_rowmax_reduce, dim3((g.nf + 63) / 64, nt), dim3(1024), 0, st,
                           (const unsigned *)p->rowpart, g.Nz * g.N, nt, g.nf, skip, p->xmax);
        LAUNCH_CHECK("k_rowmax_reduce");
    }
    int kchunk = 0;
    (void)contraction_split(p, &kchunk);
    if (p->split)
        kchunk = (kchunk + 31) / 32 * 32;
    const int split2 = (g.KK + kchunk - 1) / kchunk;
    const int fcb = p->split ? p->hfwd_cb : p->fwd_cb;
    // (the split kernel converts its A fragments with at least 5 waves)
    const int nwaves = std::max((g.NNm / 16 + fcb - 1) / fcb, p->split ? 5 : 1);
    const dim3 grid(unique_freqs(g.Q), split2, (nt + 15) / 16);
    const dim3 block(64 * nwaves);
    if (p->prof) {
        int rc = prof_event(p, 0, st);
        if (rc)
            return rc;
    }
    bool launched = false;
    if (p->split) {
#define LFRL_HFWD_LAUNCH(PT, CBV, UV)                                                            \
    hipLaunchKernelGGL((k_contract_fwd_split<PT, CBV, UV>), grid, block, 0, st,                  \
                       (const cplx16<PT::S> *)p->Hf, (const float2 *)p->X,                       \
                       (const unsigned *)p->xmax, (const int *)p->gexp, p->Yp, g.NN, g.NNm,     \
                       g.KK, g.KKs, g.KKs / 32, nt, g.nf, kchunk, skip, freq_map(g.Q),          \
                       (const float2 *)(p->Gx ? p->Gx : (float2 *)p->X), g.xcol)
#define LFRL_HFWD_CASE(CBV, UV)                                                                  \
    if (p->hfwd_cb == CBV && p->hfwd_u == UV) {                                                  \
        if (p->bf16)                                                                             \
            LFRL_HFWD_LAUNCH(PrecBF16, CBV, UV);                                                 \
        else                                                                                     \
            LFRL_HFWD_LAUNCH(PrecF16, CBV, UV);                                                  \
        launched = true;                                                                         \
    }
        LFRL_HFWD_CASE(1, 1) LFRL_HFWD_CASE(1, 2) LFRL_HFWD_CASE(2, 1) LFRL_HFWD_CASE(2, 2)
        LFRL_HFWD_CASE(3, 1)
#undef LFRL_HFWD_CASE
#undef LFRL_HFWD_LAUNCH
    } else {
    LFRL_FWD_CASES(2) LFRL_FWD_CASES(3) LFRL_FWD_CASE(4, 1) LFRL_FWD_CASE(4, 2)
    LFRL_FWD_CASE(5, 1) LFRL_FWD_CASE(5, 2)
    }
    if (!launched)
        return set_error(LFRL_ERR_UNSUPPORTED, "no forward contraction for shape %d/%d",
                         p->fwd_cb, p->fwd_u);
    LAUNCH_CHECK("k_contract_fwd");
    if (p->prof) {
        int rc = prof_event(p, 0, st);
        if (rc)
            return rc;
    }
    // partials Yp[s][k][t][c]
    const size_t sk = (size_t)g.NN * nt, split_stride = (size_t)g.nf * sk;
    if (p->use_fft)
        launch_c2r_fft(g.Q, dim3(nt * g.N), p->thr_c2r, p->lds_c2r_bytes, st, batch, p->Yp,
                       split_stride, split2, sk, g.NN, 1, g.N, 1, g.T, g.hD, p->tw,
                       p->c2r_stage);
    else
        hipLaunchKernelGGL(k_c2r, dim3(nt, g.N), dim3(256), p->lds_c2r_bytes, st, batch, p->Yp,
                           split_stride, split2, sk, (size_t)g.NN, (size_t)1, g.N, g.Q, g.QH, g.T,
                           g.hD, p->tw);
    LAUNCH_CHECK("k_c2r(forward)");
    return LFRL_OK;
}

// Back projection of n frames in one pass: img [h][w] -> vol [Nz][h][w] per
// frame, stored (STORE) or applied as the RL update
// dst = x_old * A^T img / sens (UPDATE, x_old = aux0, sens = aux1).
static int run_backward(lfrl_plan_s *p, const FrameIO *io, int n, int mode, hipStream_t st)
{
    const Geo &g = p->g;
    TileBatch batch;
    const int nt = make_batch(g, io, n, mode, &batch);
    if (nt > p->max_tiles)
        return set_error(LFRL_ERR_ARG, "batch of %d tiles exceeds the plan capacity %d", nt,
                         p->max_tiles);
    const int *skip = n == 1 ? io[0].skip : nullptr;
    if (p->use_fft)
        launch_r2c_fft(g.Q, dim3(nt * g.N), p->thr_r2c, p->lds_r2c_vol_bytes, st, SRC_PLANES, batch,
                       nullptr, g.N, g.T, g.hD, nt, g.NN, g.K, g.c0, g.KK, p->Rs, p->tw,
                       p->split ? p->rowpart : nullptr);
    else
        hipLaunchKernelGGL(k_vol_r2c, dim3(nt, g.N), dim3(256), p->lds_r2c_bytes, st, batch, g.N,
                           g.Q, g.QH, g.T, g.hD, nt, g.NN, p->Rs, p->tw);
    LAUNCH_CHECK("k_vol_r2c(image)");
    if (p->split) {
        hipLaunchKernelGGL(k_rowmax_reduce, dim3((g.nf + 63) / 64, nt), dim3(1024), 0, st,
                           (const unsigned *)p->rowpart, g.N, nt, g.nf, skip, p->rmax);
        LAUNCH_CHECK("k_rowmax_reduce");
    }
    // the back-projected tile spectra B, frequency-major [k][t][KKs] (measured
    // no faster tile-major)
    const size_t osk = (size_t)g.KKs * nt, ost = (size_t)g.KKs;
    const int acb = p->split ? p->hadj_cb : p->adj_cb;
    const int kk_per_range = 16 * acb * kAdjWaves;
    const int nrange = (g.KK + kk_per_range - 1) / kk_per_range;
    // each block stages R once and covers `ranges` kk ranges, as many as keep
    // about 2048 blocks in the launch (at most 4)
    const long long blocks1 = (long long)unique_freqs(g.Q) * nrange * ((nt + 15) / 16);
    const int ranges = (int)std::max(1LL, std::min(4LL, blocks1 / 2048));
    const dim3 grid(unique_freqs(g.Q), (nrange + ranges - 1) / ranges, (nt + 15) / 16);
    // FP32: rows of R staged in LDS, an even number of register groups of
    // 8 * adj_u reduction indices (as the kernel assumes), row stride kRsStride
    const int ustep = 8 * p->adj_u;
    const int agroups = ((g.NCm + ustep - 1) / ustep + 1) / 2 * 2;
    // split: 16-c chunks of hi/lo R values, 2 KB each (split_adj_chunks)
    const size_t lds = p->split ? (size_t)split_adj_chunks(g.NNm / 16, p->hadj_u) * 64 * 16 * 2
                                : (size_t)agroups * ustep * kRsStride * sizeof(float2);
    if (p->prof) {
        int rc = prof_event(p, 1, st);
        if (rc)
            return rc;
    }
    bool launched = false;
    if (p->split) {
#define LFRL_HADJ_LAUNCH(PT, CBV, UV)                                                            \
    hipLaunchKernelGGL((k_contract_adj_split<PT, CBV, UV>), grid, dim3(64 * kAdjWaves), lds, st, \
                       (const cplx16<PT::S> *)p->Hb, (const float2 *)p->Rs,                      \
                       (const unsigned *)p->rmax, (const int *)p->gexp, p->X, g.NN, g.NNm,      \
                       g.KK, g.KKs, (g.KK + 15) / 16, nt, skip, freq_map(g.Q),                   \
                       (const float2 *)p->Hx, g.xcol, g.KKb, osk, ost, ranges)
#define LFRL_HADJ_CASE(CBV, UV)                                                                  \
    if (p->hadj_cb == CBV && p->hadj_u == UV) {                                                  \
        if (p->bf16)                                                                             \
            LFRL_HADJ_LAUNCH(PrecBF16, CBV, UV);                                                 \
        else                                                                                     \
            LFRL_HADJ_LAUNCH(PrecF16, CBV, UV);                                                  \
        launched = true;                                                                         \
    }
        LFRL_HADJ_CASE(2, 2) LFRL_HADJ_CASE(2, 4) LFRL_HADJ_CASE(4, 2) LFRL_HADJ_CASE(4, 4)
#undef LFRL_HADJ_CASE
#undef LFRL_HADJ_LAUNCH
    } else {
    LFRL_ADJ_CASES(2) LFRL_ADJ_CASES(4)
    }
    if (!launched)
        return set_error(LFRL_ERR_UNSUPPORTED, "no adjoint contraction for shape %d/%d",
                         p->adj_cb, p->adj_u);
    LAUNCH_CHECK("k_contract_adj");
    if (p->prof) {
        int rc = prof_event(p, 1, st);
        if (rc)
            return rc;
    }
    // B, rows of KKs at k * osk + t * ost
    if (p->use_fft)
        launch_c2r_fft(g.Q, dim3(nt * g.Nz * g.N), p->thr_c2r, p->lds_c2r_bytes, st, batch, p->X,
                       (size_t)0, 1, osk, ost, 1, g.N, g.Nz, g.T, g.hD, p->tw, p->c2r_stage);
    else
        hipLaunchKernelGGL(k_c2r, dim3(nt, g.Nz * g.N), dim3(256), p->lds_c2r_bytes, st, batch,
                           p->X, (size_t)0, 1, osk, ost, (size_t)1, g.N, g.Q, g.QH, g.T,
                           g.hD, p->tw);
    LAUNCH_CHECK("k_c2r(backward)");
    return LFRL_OK;
}

// Measured choice of the tile side: for the best few sides by the model, a
// timing-only plan runs one forward and one back projection of max_batch
// largest frames (after a warm-up pair); the fastest side wins.
static int autotune_q(const lfrl_plan_desc *desc, const std::vector<int> &cands, hipStream_t st,
                      int *q_out, double *ms_out, int *tried)
{
    const int nb = std::max(1, (int)desc->max_batch);
    const size_t hw = (size_t)desc->max_h * desc->max_w, nvox = hw * desc->nz;
    float *vol = nullptr, *img = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = LFRL_OK;
    double best = 1e300;
    int bq = cands[0], n = 0;
    if ((rc = dalloc(&vol, nvox * sizeof(float))) || (rc = dalloc(&img, hw * sizeof(float))))
        goto done;
    if (hipMemsetAsync(vol, 0, nvox * sizeof(float), st) != hipSuccess ||
        hipMemsetAsync(img, 0, hw * sizeof(float), st) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = set_error(LFRL_ERR_DEVICE, "autotune set-up failed");
        goto done;
    }
    for (size_t i = 0; i < cands.size() && i < (size_t)kTuneCandidates; ++i) {
        lfrl_plan_s *tp = nullptr;
        rc = plan_build(&tp, desc, cands[i], nullptr, st);
        if (rc == LFRL_ERR_NOMEM) {  // this side does not fit: try the next
            rc = LFRL_OK;
            continue;
        }
        if (rc)
            goto done;
        FrameIO fw[kMaxBatchJobs], bw[kMaxBatchJobs];
        for (int b = 0; b < nb; ++b) {
            fw[b] = FrameIO{desc->max_h, desc->max_w, vol, img, nullptr, nullptr};
            bw[b] = FrameIO{desc->max_h, desc->max_w, img, vol, nullptr, nullptr};
        }
        float ms = 0.f;
        for (int rep = 0; rep < 3 && rc == LFRL_OK; ++rep) {
            if (rep == 1 && hipEventRecord(e0, st) != hipSuccess)
                rc = set_error(LFRL_ERR_DEVICE, "hipEventRecord failed");
            if (!rc)
                rc = run_forward(tp, fw, nb, EPI_STORE, st);
            if (!rc)
                rc = run_backward(tp, bw, nb, EPI_STORE, st);
        }
        if (!rc && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = set_error(LFRL_ERR_DEVICE, "autotune timing failed");
        free_plan(tp);
        if (rc)
            goto done;
        ++n;
        if (ms / 2.0 < best) {
            best = ms / 2.0;
            bq = cands[i];
        }
    }
    if (n == 0)
        rc = set_error(LFRL_ERR_NOMEM, "no tile size fits in device memory");
done:
    if (vol)
        (void)hipFree(vol);
    if (img)
        (void)hipFree(img);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    *q_out = bq;
    *ms_out = n ? best : 0.0;
    *tried = n;
    return rc;
}

static int launch_fill(float *ptr, size_t n, float v, hipStream_t st)
{
    const int blocks = (int)std::min<size_t>(4096, (n + 255) / 256 + 1);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, st, ptr, n, v);
    LAUNCH_CHECK("k_fill");
    return LFRL_OK;
}

static int legs_count(double legs, int n)
{
    const double c = std::ceil(legs);
    return (int)std::min<double>((double)n, c);
}

// Scratch of one metric evaluation.
struct MetricBufs {
    float *mip;
    double *tabH, *tabW, *T1, *n2p, *Fabs;
    int *tab_h, *tab_nv, *tab_w, *tab_nu;  // cached table shapes (may be null: rebuild)
};

// Area of a metric region (the entropy's prefactor is its inverse).
static double region_area(int region, double xs, double ys, int h, int w)
{
    return region == LFRL_REGION_TRIANGLE ? 0.5 * xs * ys
           : region == LFRL_REGION_RECTANGLE ? xs * ys
                                             : (double)h * (double)w;
}

// Limits of the one-block metric (k_metric_small): image pixels, row-transform
// values and candidate coefficients held in LDS (44 KB at most), and the
// volume size up to which that block also copies the best iterate.
// Launch shape of the multi-block spectral norm for an h x w image (nb = 0:
// the one-block kernel instead).  Rows of the image are spread over at most
// kSpecMaxBlocks blocks of 1024 threads, each holding its rows in LDS next to
// 3 w doubles of vectors and its row sums; the exchange needs
// spectral_mb_words(nb, w) 64-bit words of T1.
static constexpr int kSpecMaxBlocks = 32;
static constexpr size_t kSpecLds = 120 * 1024;
static constexpr size_t kSpecMinPixels = 16384;
struct SpectralLaunch {
    int nb, rpb, steps;
    size_t lds;
};
static SpectralLaunch spectral_launch(int h, int w, size_t t1cap)
{
    SpectralLaunch sp{};
    if ((size_t)h * w < kSpecMinPixels)
        return sp;
    // per row: w floats in LDS, its y value and at most 1024 / rpb + 1 pieces
    const size_t vec = (size_t)3 * w * sizeof(double) + 1024 * sizeof(double);
    const size_t per_row = (size_t)w * sizeof(float) + 2 * sizeof(double);
    if (vec + per_row > kSpecLds)
        return sp;
    const int rmax = (int)((kSpecLds - vec) / per_row);
    const int nb = (h + rmax - 1) / rmax;
    if (nb > kSpecMaxBlocks)
        return sp;
    const int rpb = (h + nb - 1) / nb;
    if (t1cap < spectral_mb_words(nb, w))
        return sp;
    const size_t steps = kLanczosMaxSteps;
    sp.nb = nb;
    sp.rpb = rpb;
    sp.steps = (int)steps;
    sp.lds = ((size_t)3 * w + spectral_mb_pieces(rpb, w) + rpb) * sizeof(double) +
             (size_t)rpb * w * sizeof(float);
    return sp;
}

static constexpr int kSmallMetricPixels = 8192;
static constexpr int kSmallMetricRows = 1024;
static constexpr int kSmallMetricCoefs = 512;
static constexpr size_t kSmallCopyVoxels = 65536;
// Spectral norm: the image size its one block holds (two float64 vectors of h
// and w in LDS).
static constexpr int kSpectralMaxSides = 6144;

// Row chunks of the leg-limited row transform: chunks of about 16 rows, as
// many as T1 holds (kMetricChunks blocks of min(h, kMaxMetricLegs) x w
// doubles), folded into the first before the column pass.
static void metric_row_chunks(int h, int nv, int *rows_per_chunk, int *nchunks)
{
    const int cap = kMetricChunks * std::min(h, kMaxMetricLegs) / nv;
    const int chunks = std::max(1, std::min((h + 15) / 16, cap));
    const int rpc = (h + chunks - 1) / chunks;
    *rows_per_chunk = rpc;
    *nchunks = (h + rpc - 1) / rpc;
}

// Argument check of a metric norm against the image size.
static int check_norm_size(int norm, int h, int w)
{
    if (norm == LFRL_NORM_SPECTRAL && h + w > kSpectralMaxSides)
        return set_error(LFRL_ERR_UNSUPPORTED, "spectral norm needs h + w <= %d", kSpectralMaxSides);
    return LFRL_OK;
}

// DCT entropy of the z-MIP of vol[nz][h][w] (nz = 1: the image itself) into
// out[0]; optional stop-state update for iteration k.  With best != nullptr the
// iterate vol is to be copied into best when it is the best so far: *copied
// tells whether the metric did that itself (small frames), else the caller
// launches k_cond_copy.
static int run_metric(int nz, int h, int w, const float *vol, double xs, double ys, int region,
                      int norm, double *out, const MetricBufs &mb, StopState *st_dev,
                      double *trace, int k, int patience, int window, hipStream_t st,
                      float *best = nullptr, size_t nvox = 0, bool *copied = nullptr,
                      const int *skip = nullptr)
{
    if (copied)
        *copied = false;
    const bool whole = region == LFRL_REGION_WHOLE;
    const int nv = whole ? h : legs_count(ys, h), nu = whole ? w : legs_count(xs, w);
    const bool cached = mb.tab_h && *mb.tab_h == h && *mb.tab_nv >= nv && *mb.tab_w == w &&
                        *mb.tab_nu >= nu;
    if (!cached) {
        hipLaunchKernelGGL(k_dct_table, dim3((h * nv + 255) / 256), dim3(256), 0, st, mb.tabH, h, nv);
        LAUNCH_CHECK("k_dct_table(H)");
        hipLaunchKernelGGL(k_dct_table, dim3((w * nu + 255) / 256), dim3(256), 0, st, mb.tabW, w, nu);
        LAUNCH_CHECK("k_dct_table(W)");
        if (mb.tab_h) {
            *mb.tab_h = h;
            *mb.tab_nv = nv;
            *mb.tab_w = w;
            *mb.tab_nu = nu;
        }
    }
    const size_t hw = (size_t)h * w;
    if (!whole && norm != LFRL_NORM_SPECTRAL && hw <= (size_t)kSmallMetricPixels &&
        nv * w <= kSmallMetricRows && nv * nu <= kSmallMetricCoefs) {
        const bool copy = best && nvox <= kSmallCopyVoxels;
        const size_t lds = ((size_t)nv * w + (size_t)nv * nu) * sizeof(double) + hw * sizeof(float);
        hipLaunchKernelGGL(k_metric_small, dim3(1), dim3(1024), lds, st, vol, nz, h, w,
                           (const double *)mb.tabH, (const double *)mb.tabW, nv, nu, xs, ys,
                           region, norm, region_area(region, xs, ys, h, w), out, st_dev, trace, k,
                           patience, std::max(1, window), copy ? best : nullptr, nvox, skip);
        LAUNCH_CHECK("k_metric_small");
        if (copied)
            *copied = copy;
        return LFRL_OK;
    }
    const int nblk = (int)((hw + 255) / 256);
    // spectral norm: sigma_1^2 of the projection into the slot after the
    // Parseval partials.  Its work space is T1 (free until the row
    // transform): at least kMetricChunks * min(h, 256) * w doubles in every
    // metric scratch.
    const size_t t1cap = std::max((size_t)kMetricChunks * std::min(h, kMaxMetricLegs) * w,
                                  (size_t)h * w);
    SpectralLaunch sp{};
    if (norm == LFRL_NORM_SPECTRAL)
        sp = spectral_launch(h, w, t1cap);
    hipLaunchKernelGGL(k_mip, dim3(nblk), dim3(256), 0, st, vol, nz, hw, mb.mip, mb.n2p, skip,
                       reinterpret_cast<unsigned long long *>(mb.T1),
                       sp.nb > 0 ? spectral_mb_words(sp.nb, w) : (size_t)0);
    LAUNCH_CHECK("k_mip");
    if (norm == LFRL_NORM_SPECTRAL) {
        if (sp.nb > 0) {
            raise_lds_attr((const void *)k_spectral_norm_mb, kSpecLds);
            hipLaunchKernelGGL(k_spectral_norm_mb, dim3(sp.nb), dim3(1024), sp.lds, st,
                               (const float *)mb.mip, h, w, sp.rpb, sp.steps,
                               reinterpret_cast<unsigned long long *>(mb.T1), skip,
                               mb.n2p + nblk);
            LAUNCH_CHECK("k_spectral_norm_mb");
        } else {
            const size_t lds = (size_t)(3 * std::min(h, w) + std::max(h, w)) * sizeof(double);
            raise_lds_attr((const void *)k_spectral_norm, 2 * kSpectralMaxSides * sizeof(double));
            hipLaunchKernelGGL(k_spectral_norm, dim3(1), dim3(1024), lds, st,
                               (const float *)mb.mip, h, w, kLanczosMaxSteps, skip, mb.n2p + nblk);
            LAUNCH_CHECK("k_spectral_norm");
        }
    }
    const int ncoef = nv * nu;
    if (whole) {
        // both passes as dense products: T1 = C_H m, |F| = |T1 C_W^T|
        hipLaunchKernelGGL((k_dgemm32<false, false, float>), dim3((w + 31) / 32, (h + 31) / 32),
                           dim3(256), 0, st, (const double *)mb.tabH, h, (const float *)mb.mip, w,
                           h, w, h, mb.T1, w);
        LAUNCH_CHECK("k_dgemm32(rows)");
        hipLaunchKernelGGL((k_dgemm32<true, true, double>), dim3((w + 31) / 32, (h + 31) / 32),
                           dim3(256), 0, st, (const double *)mb.T1, w, (const double *)mb.tabW, w,
                           h, w, w, mb.Fabs, w);
        LAUNCH_CHECK("k_dgemm32(columns)");
    } else {
        int rpc = 0, nchunks = 0;
        metric_row_chunks(h, nv, &rpc, &nchunks);
        hipLaunchKernelGGL(k_dct_rows, dim3((nv * w + 255) / 256, nchunks), dim3(256), 0, st,
                           (const float *)mb.mip, h, w, (const double *)mb.tabH, nv, rpc, mb.T1);
        LAUNCH_CHECK("k_dct_rows");
        if (nchunks > 1) {
            hipLaunchKernelGGL(k_dct_fold, dim3((nv * w + 255) / 256), dim3(256), 0, st, mb.T1,
                               nchunks, nv * w);
            LAUNCH_CHECK("k_dct_fold");
        }
        hipLaunchKernelGGL(k_metric_coeffs, dim3((ncoef + 3) / 4), dim3(256), 0, st,
                           (const double *)mb.T1, 1, nv, nu, w, (const double *)mb.tabW, xs, ys,
                           region, mb.Fabs);
        LAUNCH_CHECK("k_metric_coeffs");
    }
    // large coefficient sets: the entropy sum over many blocks, its partials in
    // T1 (free once the coefficients are formed; it holds >= 8 * 16384 doubles)
    const double *ent = nullptr;
    int nent = 0;
    if (ncoef > kMetricBigCoefs) {
        double *sq = mb.T1, *part = mb.T1 + kDotBlocks;
        const double *n2src = mb.n2p;
        int n2count = nblk;
        if (norm == LFRL_NORM_SPECTRAL) {
            n2src = mb.n2p + nblk;
            n2count = 1;
        } else if (norm == LFRL_NORM_REGION) {
            hipLaunchKernelGGL(k_sq_partial, dim3(kDotBlocks), dim3(256), 0, st,
                               (const double *)mb.Fabs, ncoef, sq);
            LAUNCH_CHECK("k_sq_partial");
            n2src = sq;
            n2count = kDotBlocks;
        }
        hipLaunchKernelGGL(k_entropy_partial, dim3(kDotBlocks), dim3(256), 0, st, n2src, n2count,
                           (const double *)mb.Fabs, ncoef, part);
        LAUNCH_CHECK("k_entropy_partial");
        ent = part;
        nent = kDotBlocks;
    }
    hipLaunchKernelGGL(k_metric_final, dim3(1), dim3(256), 0, st, (const double *)mb.n2p, nblk,
                       (const double *)mb.Fabs, ncoef, norm, region_area(region, xs, ys, h, w),
                       out, st_dev, trace, k, patience, std::max(1, window), ent, nent, skip);
    LAUNCH_CHECK("k_metric_final");
    return LFRL_OK;
}

static int check_legs(double xs, double ys, int region = LFRL_REGION_TRIANGLE)
{
    if (region == LFRL_REGION_WHOLE)
        return LFRL_OK;
    if (!(xs > 0.0) || !(ys > 0.0) || !std::isfinite(xs) || !std::isfinite(ys))
        return set_error(LFRL_ERR_ARG, "triangle legs xs=%g, ys=%g must be positive", xs, ys);
    if (std::ceil(xs) > kMaxMetricLegs || std::ceil(ys) > kMaxMetricLegs)
        return set_error(LFRL_ERR_UNSUPPORTED, "triangle legs above %d bins", kMaxMetricLegs);
    return LFRL_OK;
}

static MetricBufs frame_metric_bufs(Frame &f)
{
    return MetricBufs{f.mip, f.tabH, f.tabW, f.T1, f.n2p, f.Fabs,
                      &f.tab_h, &f.tab_nv, &f.tab_w, &f.tab_nu};
}

// c = A^T 1 for the frame's image size, through the tile-DFT path, then made
// exact (float64 window sums) at the weakly observed voxels, which are listed
// for the per-iteration fix-up.  With check_input, the frame's image is also
// checked for negative or non-finite values (LFRL_ERR_NUMERIC).  Synchronises
// the stream.
static int frame_sensitivity(lfrl_plan_s *p, Frame &f, bool check_input, hipStream_t st)
{
    const int h = f.h, w = f.w;
    const size_t hw = (size_t)h * w, nvox = (size_t)p->g.Nz * hw;
    f.nweak = 0;
    int rc = launch_fill(f.rho, hw, 1.0f, st);
    if (rc)
        return rc;
    const FrameIO io{h, w, f.rho, f.sens, nullptr, nullptr};
    rc = run_backward(p, &io, 1, EPI_STORE, st);
    if (rc)
        return rc;
    hipLaunchKernelGGL(k_max_partial, dim3(kDotBlocks), dim3(256), 0, st, (const float *)f.sens,
                       nvox, f.cmax);
    LAUNCH_CHECK("k_max_partial");
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, st, (const float *)f.cmax, kDotBlocks,
                       f.cmax + kDotBlocks, f.counters);
    LAUNCH_CHECK("k_max_final");
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, f.counters + 1);
    LAUNCH_CHECK("k_zero_u32");
    if (check_input) {
        hipLaunchKernelGGL(k_check_image, dim3(256), dim3(256), 0, st, f.y, hw, f.counters + 1);
        LAUNCH_CHECK("k_check_image");
    }
    float thr = kWeakThreshold, used = thr;
    unsigned found = 0;
    for (int attempt = 0; attempt < 8; ++attempt) {
        used = thr;
        if (attempt > 0) {
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, f.counters);
            LAUNCH_CHECK("k_zero_u32");
        }
        hipLaunchKernelGGL(k_weak_select, dim3(2048), dim3(256), 0, st, (const float *)f.sens,
                           nvox, (const float *)(f.cmax + kDotBlocks), thr, f.weak, f.counters,
                           f.weak_cap);
        LAUNCH_CHECK("k_weak_select");
        HIP_TRY(hipMemcpyAsync(f.counters_host, f.counters, 2 * sizeof(unsigned),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        found = f.counters_host[0];
        if (found <= f.weak_cap)
            break;
        thr *= 0.1f;
    }
    if (check_input && f.counters_host[1])
        return set_error(LFRL_ERR_NUMERIC, "image has negative or non-finite values");
    if (found > f.weak_cap)
        // a partial list would leave some weak voxels on the inexact path, and
        // which ones would depend on the order of the atomic appends
        return set_error(LFRL_ERR_UNSUPPORTED,
                         "%u weakly observed voxels (A^T 1 below %g of its maximum) exceed the "
                         "list of %u",
                         found, (double)used, f.weak_cap);
    f.nweak = found;
    if (f.nweak) {
        hipLaunchKernelGGL(k_weak_exact, dim3(f.nweak), dim3(kWeakThreads), 0, st, (const unsigned *)f.weak,
                           (const float *)p->psf, p->g.N, p->g.K, h, w, (const float *)nullptr,
                           f.sens, (const float *)nullptr, (const float *)nullptr, (float *)nullptr,
                           (int)WEAK_SENS, (const int *)nullptr);
        LAUNCH_CHECK("k_weak_exact(sens)");
    }
    return LFRL_OK;
}

// Sensitivity of the plan's own frame, cached per image size.
static int ensure_sensitivity(lfrl_plan_s *p, int h, int w, hipStream_t st)
{
    if (p->sens_h == h && p->sens_w == w)
        return LFRL_OK;
    p->sens_h = p->sens_w = -1;
    p->fr.h = h;
    p->fr.w = w;
    int rc = frame_sensitivity(p, p->fr, false, st);
    if (rc)
        return rc;
    p->sens_h = h;
    p->sens_w = w;
    return LFRL_OK;
}

// Float64 sum(a * b) (b == nullptr: sum(a)) into the frame's stop state
// (which = 0: the image sum) or its flux trace at iteration k (which = 1).
static int frame_dot(Frame &f, const float *a, const float *b, size_t n, int k, int which,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, st, a, b, n, f.dotp);
    LAUNCH_CHECK("k_dot_partial");
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, (const double *)f.dotp, kDotBlocks,
                       f.state, f.flux, k, which);
    LAUNCH_CHECK("k_dot_final");
    return LFRL_OK;
}

static int check_opts(const lfrl_rl_opts *opts)
{
    if (opts->max_iters < 1 || opts->max_iters > kMaxTrace)
        return set_error(LFRL_ERR_ARG, "max_iters must be in [1, %d]", kMaxTrace);
    if (opts->stop < LFRL_STOP_NONE || opts->stop > LFRL_STOP_TRACK)
        return set_error(LFRL_ERR_ARG, "unknown stop mode %d", opts->stop);
    if (opts->init < 0 || opts->init > 2)
        return set_error(LFRL_ERR_ARG, "init must be 0, 1 or 2");
    if (opts->update != LFRL_UPDATE_RL && opts->update != LFRL_UPDATE_ISRA)
        return set_error(LFRL_ERR_ARG, "unknown update rule %d", opts->update);
    if (!(opts->background >= 0.0) || !(opts->background <= 3.4e38))
        return set_error(LFRL_ERR_ARG, "background must be finite and >= 0");
    if (opts->stop != LFRL_STOP_NONE) {
        if (opts->patience < 1)
            return set_error(LFRL_ERR_ARG, "patience must be >= 1");
        if (opts->window < 0 || opts->window > kMaxTrace)
            return set_error(LFRL_ERR_ARG, "window must be in [0, %d]", kMaxTrace);
        if (opts->region < LFRL_REGION_TRIANGLE || opts->region > LFRL_REGION_WHOLE)
            return set_error(LFRL_ERR_ARG, "unknown metric region %d", opts->region);
        if (opts->norm < LFRL_NORM_MATRIX || opts->norm > LFRL_NORM_SPECTRAL)
            return set_error(LFRL_ERR_ARG, "unknown metric norm %d", opts->norm);
        return check_legs(opts->xs, opts->ys, opts->region);
    }
    return LFRL_OK;
}

// D = A^T y for the ISRA numerator and the back projection start, with the
// weakly observed voxels' window sums in float64.
static int frame_backproject_image(lfrl_plan_s *p, Frame &f, hipStream_t st)
{
    const FrameIO io{f.h, f.w, f.y, f.D, nullptr, nullptr};
    int rc = run_backward(p, &io, 1, EPI_STORE, st);
    if (rc)
        return rc;
    if (f.nweak) {
        hipLaunchKernelGGL(k_weak_exact, dim3(f.nweak), dim3(kWeakThreads), 0, st, (const unsigned *)f.weak,
                           (const float *)p->psf, p->g.N, p->g.K, f.h, f.w, f.y, f.sens,
                           (const float *)nullptr, (const float *)nullptr, f.D, (int)WEAK_STORE,
                           (const int *)nullptr);
        LAUNCH_CHECK("k_weak_exact(store)");
    }
    return LFRL_OK;
}

// x^0 (ones, a copy of vol0, or A^T y), A^T y when the ISRA update needs it, a
// fresh stop state, and the image sum for the flux trace.  Needs A^T 1 and
// the weak-voxel list of the frame.
static int frame_start(lfrl_plan_s *p, Frame &f, const float *vol0, hipStream_t st)
{
    const size_t nvox = (size_t)p->g.Nz * f.h * f.w;
    if (f.opts.update == LFRL_UPDATE_ISRA || f.opts.init == 2) {
        int rc = frame_backproject_image(p, f, st);
        if (rc)
            return rc;
    }
    if (f.opts.init == 2) {
        HIP_TRY(hipMemcpyAsync(f.V[0], f.D, nvox * sizeof(float), hipMemcpyDeviceToDevice, st));
    } else if (vol0) {
        HIP_TRY(hipMemcpyAsync(f.V[0], vol0, nvox * sizeof(float), hipMemcpyDeviceToDevice, st));
    } else {
        int rc = launch_fill(f.V[0], nvox, 1.0f, st);
        if (rc)
            return rc;
    }
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1), 0, st, f.state);
    LAUNCH_CHECK("k_state_reset");
    if (f.want_flux) {
        int rc = frame_dot(f, f.y, nullptr, (size_t)f.h * f.w, 0, 0, st);
        if (rc)
            return rc;
    }
    f.iters = 0;
    f.done = f.stopped = false;
    return LFRL_OK;
}

// One iteration for n frames of plan p, their projections batched (each
// frame with its own update rule and background b):
//   RL:   rho = y / (A x^{k-1} + b),  x^k = x^{k-1} * A^T rho / c;
//   ISRA: rho = A x^{k-1} + b,        x^k = x^{k-1} * A^T y / A^T rho;
// the exact update at the weakly observed voxels, then the metric,
// best-iterate copy and flux of each frame.  Queued on `st` without
// synchronising.
// Device flag that turns a frame's later iterations into no-ops once its stop
// rule has fired (early-stop mode only: several iterations may then be queued
// before the host reads the decision).  Null otherwise.
static const int *frame_skip(const Frame &f)
{
    return f.opts.stop == LFRL_STOP_METRIC ? &f.state->stopped : nullptr;
}

static int step_frames(lfrl_plan_s *p, Frame *const *fr, int n, hipStream_t st)
{
    FrameIO io[kMaxBatchJobs];
    for (int i = 0; i < n; ++i) {
        Frame &f = *fr[i];
        const int k = f.iters + 1;
        const bool isra = f.opts.update == LFRL_UPDATE_ISRA;
        io[i] = FrameIO{f.h, f.w, f.V[(k - 1) & 1], f.rho, f.y, nullptr,
                        (float)f.opts.background, isra ? EPI_STORE : EPI_RATIO, frame_skip(f)};
    }
    int rc = run_forward(p, io, n, EPI_RATIO, st);
    if (rc)
        return rc;
    for (int i = 0; i < n; ++i) {
        Frame &f = *fr[i];
        const int k = f.iters + 1;
        const bool isra = f.opts.update == LFRL_UPDATE_ISRA;
        io[i] = FrameIO{f.h, f.w, f.rho, f.V[k & 1], f.V[(k - 1) & 1], isra ? f.D : f.sens,
                        0.f, isra ? EPI_ISRA : EPI_UPDATE, frame_skip(f)};
    }
    rc = run_backward(p, io, n, EPI_UPDATE, st);
    if (rc)
        return rc;
    for (int i = 0; i < n; ++i) {
        Frame &f = *fr[i];
        const int k = f.iters + 1;
        const float *cur = f.V[(k - 1) & 1];
        float *nxt = f.V[k & 1];
        const size_t nvox = (size_t)p->g.Nz * f.h * f.w;
        if (f.nweak) {
            const bool isra = f.opts.update == LFRL_UPDATE_ISRA;
            hipLaunchKernelGGL(k_weak_exact, dim3(f.nweak), dim3(kWeakThreads), 0, st,
                               (const unsigned *)f.weak, (const float *)p->psf, p->g.N, p->g.K,
                               f.h, f.w, (const float *)f.rho, f.sens, cur, (const float *)f.D,
                               nxt, (int)(isra ? WEAK_ISRA : WEAK_UPDATE), frame_skip(f));
            LAUNCH_CHECK("k_weak_exact(update)");
        }
        if (f.opts.stop != LFRL_STOP_NONE) {
            bool copied = false;
            rc = run_metric(p->g.Nz, f.h, f.w, nxt, f.opts.xs, f.opts.ys, f.opts.region,
                            f.opts.norm, f.metric_out, frame_metric_bufs(f), f.state, f.trace, k,
                            f.opts.patience, f.opts.window, st, f.VB, nvox, &copied,
                            frame_skip(f));
            if (rc)
                return rc;
            if (!copied) {
                hipLaunchKernelGGL(k_cond_copy, dim3(1024), dim3(256), 0, st,
                                   (const StopState *)f.state, (const float *)nxt, f.VB, nvox);
                LAUNCH_CHECK("k_cond_copy");
            }
        }
        if (f.want_flux) {
            rc = frame_dot(f, f.sens, nxt, nvox, k, 1, st);
            if (rc)
                return rc;
        }
        f.iters = k;
    }
    return LFRL_OK;
}

// After a step: queue the copy of the stop state a METRIC frame needs.
static int frame_queue_poll(Frame &f, hipStream_t st)
{
    if (f.opts.stop == LFRL_STOP_METRIC)
        HIP_TRY(hipMemcpyAsync(f.state_host, f.state, sizeof(StopState), hipMemcpyDeviceToHost, st));
    return LFRL_OK;
}

// After the stream has reached the polled state: the frame is done at the cap
// or once the stop rule fired.
static void frame_update_done(Frame &f)
{
    if (f.opts.stop == LFRL_STOP_METRIC && f.state_host->stopped)
        f.stopped = true;
    f.done = f.stopped || f.iters >= f.opts.max_iters;
}

// Copy x^{best} (metric modes) or the last iterate into vol, and fill the
// report.  Synchronises the stream.
static int frame_result(Frame &f, int nz, float *vol, lfrl_rl_report *report, hipStream_t st)
{
    const size_t nvox = (size_t)nz * f.h * f.w;
    const bool use_metric = f.opts.stop != LFRL_STOP_NONE;
    int best = f.iters;
    if (use_metric) {
        HIP_TRY(hipMemcpyAsync(f.state_host, f.state, sizeof(StopState), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        best = f.state_host->best_k;
    }
    if (vol && f.iters > 0)
        HIP_TRY(hipMemcpyAsync(vol, use_metric ? f.VB : f.V[f.iters & 1], nvox * sizeof(float),
                               hipMemcpyDeviceToDevice, st));
    else if (vol)
        HIP_TRY(hipMemcpyAsync(vol, f.V[0], nvox * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (report && f.iters > 0) {
        if (use_metric && report->metric_trace)
            HIP_TRY(hipMemcpyAsync(report->metric_trace, f.trace, f.iters * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
        if (f.want_flux && report->flux_trace)
            HIP_TRY(hipMemcpyAsync(report->flux_trace, f.flux, f.iters * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    if (report) {
        report->iters_run = f.iters;
        report->best_iter = best;
        report->stopped = f.stopped ? 1 : 0;
        report->weak_voxels = (int32_t)f.nweak;
    }
    return LFRL_OK;
}

// ---------------------------------------------------------------------------
// public entry points
// ---------------------------------------------------------------------------
extern "C" int lfrl_forward(lfrl_plan_t p, int32_t h, int32_t w, const float *vol, float *img,
                            void *stream)
{
    if (!p || !vol || !img)
        return set_error(LFRL_ERR_ARG, "NULL argument");
    int rc = check_hw(p, h, w);
    if (rc)
        return rc;
    DevGuard dg(p->device);
    const size_t npx = (size_t)h * w;
    if ((rc = check_buf(vol, npx * p->g.Nz * sizeof(float), "vol")) ||
        (rc = check_buf(img, npx * sizeof(float), "img")))
        return rc;
    const FrameIO io{h, w, vol, img, nullptr, nullptr};
    return run_forward(p, &io, 1, EPI_STORE, (hipStream_t)stream);
}

extern "C" int lfrl_backward(lfrl_plan_t p, int32_t h, int32_t w, const float *img, float *vol,
                             void *stream)
{
    if (!p || !vol || !img)
        return set_error(LFRL_ERR_ARG, "NULL argument");
    int rc = check_hw(p, h, w);
    if (rc)
        return rc;
    DevGuard dg(p->device);
    const size_t npx = (size_t)h * w;
    if ((rc = check_buf(vol, npx * p->g.Nz * sizeof(float), "vol")) ||
        (rc = check_buf(img, npx * sizeof(float), "img")))
        return rc;
    const FrameIO io{h, w, img, vol, nullptr, nullptr};
    return run_backward(p, &io, 1, EPI_STORE, (hipStream_t)stream);
}

// Early-stop runs (sec. 2.2: stop once the entropy decreases) queue their
// iterations in chunks of kStopChunk; the host reads the stop state of a chunk
// while the next one is already queued.  Every kernel of a frame's iteration
// returns at once when the frame's stop flag was raised by an earlier
// iteration, so iterations queued past the stop change nothing and the result
// equals a run that looks at the rule after every iteration.  With graphs
// allowed, each chunk is captured once (keyed like the fixed-length graph,
// plus its first iteration) and replayed.
static constexpr int kStopChunk = 4;
static constexpr size_t kMaxChunkGraphs = 64;   // chunk graphs kept per plan

static int launch_stop_chunk(lfrl_plan_s *p, Frame &f, int k0, float *vol0, bool graphs,
                             hipStream_t st)
{
    const int k1 = std::min(f.opts.max_iters, k0 + kStopChunk);
    Frame *one[1] = {&f};
    if (!graphs) {
        int rc = LFRL_OK;
        if (k0 == 0)
            rc = frame_start(p, f, vol0, st);
        f.iters = k0;
        while (rc == LFRL_OK && f.iters < k1)
            rc = step_frames(p, one, 1, st);
        return rc;
    }
    for (auto &c : p->chunk_graphs)
        if (c.k0 == k0) {
            ++p->graph_hits;
            HIP_TRY(hipGraphLaunch(c.exec, st));
            f.iters = k1;
            return LFRL_OK;
        }
    if (p->chunk_graphs.size() >= kMaxChunkGraphs)   // very long runs: launch the rest directly
        return launch_stop_chunk(p, f, k0, vol0, false, st);
    if (!p->cap_stream)
        HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    // the captured chunk builds its own DCT tables
    f.tab_h = f.tab_nv = f.tab_w = f.tab_nu = -1;
    HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = LFRL_OK;
    if (k0 == 0)
        rc = frame_start(p, f, vol0, p->cap_stream);
    f.iters = k0;
    while (rc == LFRL_OK && f.iters < k1)
        rc = step_frames(p, one, 1, p->cap_stream);
    hipGraph_t gr = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->cap_stream, &gr);
    if (rc) {
        if (gr)
            (void)hipGraphDestroy(gr);
        return rc;
    }
    if (ec != hipSuccess)
        return set_error(LFRL_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(ec));
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(gr);
        return set_error(LFRL_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    p->chunk_graphs.push_back({k0, gr, ex});
    f.tab_h = f.tab_nv = f.tab_w = f.tab_nu = -1;
    HIP_TRY(hipGraphLaunch(ex, st));
    return LFRL_OK;
}

static int deconvolve_early_stop(lfrl_plan_s *p, Frame &f, int h, int w, const float *img,
                                 float *vol, const lfrl_rl_opts *opts, lfrl_rl_report *report,
                                 hipStream_t st, bool graphs)
{
    if (graphs) {
        const lfrl_plan_s::GraphKey key{h, w, opts->max_iters, opts->stop, opts->patience,
                                        opts->init, f.want_flux ? 1 : 0, opts->update,
                                        opts->region, opts->norm, opts->window, opts->xs,
                                        opts->ys, opts->background, img, vol};
        if (!(p->chunk_key == key)) {
            for (auto &c : p->chunk_graphs) {
                (void)hipGraphExecDestroy(c.exec);
                (void)hipGraphDestroy(c.graph);
            }
            p->chunk_graphs.clear();
            p->chunk_key = key;
        }
    }
    for (hipEvent_t &e : p->chunk_ev)
        if (!e)
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    float *vol0 = opts->init == 1 ? vol : nullptr;
    int k0 = 0, slot = 0;
    int rc = launch_stop_chunk(p, f, k0, vol0, graphs, st);
    if (rc)
        return rc;
    HIP_TRY(hipMemcpyAsync(&f.state_host[slot], f.state, sizeof(StopState), hipMemcpyDeviceToHost,
                           st));
    HIP_TRY(hipEventRecord(p->chunk_ev[slot], st));
    for (;;) {
        const int next = k0 + kStopChunk;
        const bool more = next < opts->max_iters;
        if (more) {
            // queue the next chunk before looking at this one's decision
            if ((rc = launch_stop_chunk(p, f, next, vol0, graphs, st)))
                return rc;
            HIP_TRY(hipMemcpyAsync(&f.state_host[1 - slot], f.state, sizeof(StopState),
                                   hipMemcpyDeviceToHost, st));
            HIP_TRY(hipEventRecord(p->chunk_ev[1 - slot], st));
        }
        HIP_TRY(hipEventSynchronize(p->chunk_ev[slot]));
        const StopState &ss = f.state_host[slot];
        if (ss.stopped) {
            f.iters = ss.stop_k;
            f.stopped = true;
            break;
        }
        if (!more) {
            f.iters = opts->max_iters;
            f.stopped = false;
            break;
        }
        k0 = next;
        slot = 1 - slot;
    }
    f.done = true;
    return frame_result(f, p->g.Nz, vol, report, st);
}

extern "C" int lfrl_deconvolve(lfrl_plan_t p, int32_t h, int32_t w, const float *img, float *vol,
                               const lfrl_rl_opts *opts, lfrl_rl_report *report, void *stream)
{
    if (!p || !img || !vol || !opts)
        return set_error(LFRL_ERR_ARG, "NULL argument");
    int rc = check_hw(p, h, w);
    if (rc)
        return rc;
    if ((rc = check_opts(opts)))
        return rc;
    if (opts->stop != LFRL_STOP_NONE && (rc = check_norm_size(opts->norm, h, w)))
        return rc;
    DevGuard dg(p->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t nvox = (size_t)p->g.Nz * h * w;
    if ((rc = check_buf(vol, nvox * sizeof(float), "vol")) ||
        (rc = check_buf(img, (size_t)h * w * sizeof(float), "img")))
        return rc;
    if ((rc = ensure_sensitivity(p, h, w, st)))
        return rc;
    Frame &f = p->fr;
    f.y = img;
    f.opts = *opts;
    f.want_flux = report && report->flux_trace;
    // Fixed-length runs (no host decision between iterations) are captured
    // once into a graph and replayed: one launch instead of a dozen per
    // iteration, which is what small frames are bound by.
    const char *genv = getenv("LFRL_GRAPH");
    const bool use_graph = opts->stop != LFRL_STOP_METRIC && !p->prof && !(genv && genv[0] == '0');
    if (use_graph) {
        const lfrl_plan_s::GraphKey key{h,
                                         w,
                                         opts->max_iters,
                                         opts->stop,
                                         opts->patience,
                                         opts->init,
                                         f.want_flux ? 1 : 0,
                                         opts->update,
                                         opts->region,
                                         opts->norm,
                                         opts->window,
                                         opts->xs,
                                         opts->ys,
                                         opts->background,
                                         img,
                                         vol};
        if (!(p->graph_exec && p->graph_key == key)) {
            if (p->graph_exec)
                (void)hipGraphExecDestroy(p->graph_exec);
            if (p->graph)
                (void)hipGraphDestroy(p->graph);
            p->graph_exec = nullptr;
            p->graph = nullptr;
            if (!p->cap_stream)
                HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
            // the graph builds its own DCT tables (a later call with other legs
            // may reuse the table buffers between replays)
            f.tab_h = f.tab_nv = f.tab_w = f.tab_nu = -1;
            HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
            Frame *one[1] = {&f};
            rc = frame_start(p, f, opts->init == 1 ? vol : nullptr, p->cap_stream);
            while (rc == LFRL_OK && f.iters < opts->max_iters)
                rc = step_frames(p, one, 1, p->cap_stream);
            hipGraph_t gr = nullptr;
            const hipError_t ec = hipStreamEndCapture(p->cap_stream, &gr);
            if (rc) {
                if (gr)
                    (void)hipGraphDestroy(gr);
                return rc;
            }
            if (ec != hipSuccess)
                return set_error(LFRL_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(ec));
            p->graph = gr;
            HIP_TRY(hipGraphInstantiate(&p->graph_exec, gr, nullptr, nullptr, 0));
            p->graph_key = key;
        } else {
            ++p->graph_hits;
        }
        HIP_TRY(hipGraphLaunch(p->graph_exec, st));
        f.tab_h = f.tab_nv = f.tab_w = f.tab_nu = -1;  // the replay rewrote the tables
        f.iters = opts->max_iters;
        f.done = true;
        f.stopped = false;
        return frame_result(f, p->g.Nz, vol, report, st);
    }
    if (opts->stop == LFRL_STOP_METRIC)
        return deconvolve_early_stop(p, f, h, w, img, vol, opts, report, st, !p->prof &&
                                     !(genv && genv[0] == '0'));
    if ((rc = frame_start(p, f, opts->init == 1 ? vol : nullptr, st)))
        return rc;
    Frame *one[1] = {&f};
    while (!f.done) {
        if ((rc = step_frames(p, one, 1, st)))
            return rc;
        frame_update_done(f);
    }
    return frame_result(f, p->g.Nz, vol, report, st);
}

// ---------------------------------------------------------------------------
// jobs: batched and served deconvolution
// ---------------------------------------------------------------------------
struct lfrl_job_s {
    lfrl_plan_s *plan = nullptr;  // must outlive the job
    int device = 0;
    Frame f;
    hipEvent_t used = nullptr;    // the slot's event: recorded after each use
};

// Mark the job's work queued so far on `st` (release waits for it).
static int job_mark(lfrl_job_s *j, hipStream_t st)
{
    HIP_TRY(hipEventRecord(j->used, st));
    return LFRL_OK;
}

extern "C" int lfrl_job_footprint(lfrl_plan_t p, int32_t h, int32_t w, size_t *bytes)
{
    if (!p || !bytes)
        return set_error(LFRL_ERR_ARG, "NULL argument");
    int rc = check_hw(p, h, w);
    if (rc)
        return rc;
    size_t off[FB_COUNT];
    *bytes = job_size_class(frame_layout(p->g, h, w, true, off));
    return LFRL_OK;
}

// Return a job's block and pinned words to the pool.  Work queued on the
// job must have completed (as for lfrl_job_destroy).
static void free_job(lfrl_job_s *j)
{
    if (!j)
        return;
    if (j->f.block) {
        DevGuard dg(j->device);
        (void)hipEventSynchronize(j->used);  // queued work on the block has finished
        JobSlot s;
        s.block = j->f.block;
        s.bytes = j->f.block_bytes;
        s.state_host = j->f.state_host;
        s.counters_host = j->f.counters_host;
        s.used = j->used;
        slot_put(j->device, s);
    }
    delete j;
}

// A^T 1 of a job: copied from the plan's cache when its image size was seen
// recently, else formed (frame_sensitivity) and cached (least recently used
// sizes are dropped beyond the cache limit).  Either way the job's image is
// checked (LFRL_ERR_NUMERIC) and the stream synchronised.
static int job_sensitivity(lfrl_plan_s *p, Frame &f, hipStream_t st)
{
    const size_t hw = (size_t)f.h * f.w, nvox = (size_t)p->g.Nz * hw;
    for (auto &e : p->sens_cache) {
        if (e.h != f.h || e.w != f.w)
            continue;
        e.stamp = ++p->sens_clock;
        HIP_TRY(hipMemcpyAsync(f.sens, e.sens, nvox * sizeof(float), hipMemcpyDeviceToDevice, st));
        if (e.nweak)
            HIP_TRY(hipMemcpyAsync(f.weak, e.weak, e.nweak * sizeof(unsigned),
                                   hipMemcpyDeviceToDevice, st));
        f.nweak = e.nweak;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, f.counters + 1);
        LAUNCH_CHECK("k_zero_u32");
        hipLaunchKernelGGL(k_check_image, dim3(256), dim3(256), 0, st, f.y, hw, f.counters + 1);
        LAUNCH_CHECK("k_check_image");
        HIP_TRY(hipMemcpyAsync(f.counters_host, f.counters, 2 * sizeof(unsigned),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (f.counters_host[1])
            return set_error(LFRL_ERR_NUMERIC, "image has negative or non-finite values");
        return LFRL_OK;
    }
    int rc = frame_sensitivity(p, f, true, st);
    if (rc)
        return rc;
    const size_t bytes = nvox * sizeof(float) + (size_t)f.nweak * sizeof(unsigned);
    if (bytes > p->sens_cache_limit)
        return LFRL_OK;
    while (p->sens_cache_bytes + bytes > p->sens_cache_limit && !p->sens_cache.empty()) {
        size_t old = 0;
        for (size_t i = 1; i < p->sens_cache.size(); ++i)
            if (p->sens_cache[i].stamp < p->sens_cache[old].stamp)
                old = i;
        (void)hipStreamSynchronize(st);
        (void)hipFree(p->sens_cache[old].sens);
        (void)hipFree(p->sens_cache[old].weak);
        p->sens_cache_bytes -= p->sens_cache[old].bytes;
        p->sens_cache[old] = p->sens_cache.back();
        p->sens_cache.pop_back();
    }
    lfrl_plan_s::SensEntry e;
    e.h = f.h;
    e.w = f.w;
    e.nweak = f.nweak;
    e.bytes = bytes;
    if (hipMalloc((void **)&e.sens, nvox * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&e.weak, std::max<size_t>(1, f.nweak) * sizeof(unsigned)) != hipSuccess) {
        (void)hipGetLastError();  // no room to cache: the job itself is fine
        if (e.sens)
            (void)hipFree(e.sens);
        return LFRL_OK;
    }
    HIP_TRY(hipMemcpyAsync(e.sens, f.sens, nvox * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (f.nweak)
        HIP_TRY(hipMemcpyAsync(e.weak, f.weak, f.nweak * sizeof(unsigned), hipMemcpyDeviceToDevice,
                               st));
    e.stamp = ++p->sens_clock;
    p->sens_cache.push_back(e);
    p->sens_cache_bytes += bytes;
    return LFRL_OK;
}

extern "C" int lfrl_job_create(lfrl_job_t *out, lfrl_plan_t p, int32_t h, int32_t w,
                               const float *img, const float *vol0, const lfrl_rl_opts *opts,
                               uint32_t flags, void *stream)
{
    if (!out)
        return set_error(LFRL_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!p || !img || !opts)
        return set_error(LFRL_ERR_ARG, "NULL argument");
    int rc = check_hw(p, h, w);
    if (rc)
        return rc;
    if ((rc = check_opts(opts)))
        return rc;
    if (opts->stop != LFRL_STOP_NONE && (rc = check_norm_size(opts->norm, h, w)))
        return rc;
    if (flags & ~(uint32_t)LFRL_JOB_FLUX)
        return set_error(LFRL_ERR_ARG, "unknown job flags 0x%x", flags);
    if (opts->init == 1 && !vol0)
        return set_error(LFRL_ERR_ARG, "init = 1 needs vol0");
    DevGuard dg(p->device);
    hipStream_t st = (hipStream_t)stream;
    const size_t hw = (size_t)h * w;
    if ((rc = check_buf(img, hw * sizeof(float), "img")))
        return rc;
    if (opts->init == 1 && (rc = check_buf(vol0, hw * p->g.Nz * sizeof(float), "vol0")))
        return rc;
    lfrl_job_s *j = new lfrl_job_s();
    j->plan = p;
    j->device = p->device;
    Frame &f = j->f;
    {
        size_t off[FB_COUNT];
        const size_t need = frame_layout(p->g, h, w, true, off);
        JobSlot s;
        if ((rc = slot_get(p->device, job_size_class(need), &s))) {
            delete j;
            return rc;
        }
        f.block = s.block;
        f.block_bytes = s.bytes;
        f.state_host = s.state_host;
        f.counters_host = s.counters_host;
        j->used = s.used;
        frame_bind(f, p->g, h, w, f.block, off, true);
    }
    f.opts = *opts;
    f.want_flux = (flags & LFRL_JOB_FLUX) != 0;
    hipError_t e = hipMemcpyAsync(f.y_own, img, hw * sizeof(float), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
        free_job(j);
        return set_error(LFRL_ERR_DEVICE, "image copy failed: %s", hipGetErrorString(e));
    }
    f.y = f.y_own;
    if ((rc = job_sensitivity(p, f, st)) ||
        (rc = frame_start(p, f, opts->init == 1 ? vol0 : nullptr, st)) ||
        (rc = job_mark(j, st))) {
        const std::string msg = lfrl_last_error();
        (void)hipStreamSynchronize(st);
        free_job(j);
        set_error(rc, "%s", msg.c_str());
        return rc;
    }
    *out = j;
    return LFRL_OK;
}

// Internal streams that run the jobs of different plans side by side (default
// priority, non-blocking), one set per device.
struct StreamPool {
    std::vector<hipStream_t> s;
    std::vector<hipEvent_t> done;
    hipEvent_t fork = nullptr;
};
static constexpr int kPoolStreams = 4;
static std::mutex g_pool_mu;
static std::vector<StreamPool> g_pools;

static int get_pool(int dev, StreamPool **out)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if ((int)g_pools.size() <= dev)
        g_pools.resize(dev + 1);
    StreamPool &sp = g_pools[dev];
    if (sp.s.empty()) {
        HIP_TRY(hipEventCreateWithFlags(&sp.fork, hipEventDisableTiming));
        for (int i = 0; i < kPoolStreams; ++i) {
            hipStream_t s;
            hipEvent_t e;
            HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            sp.s.push_back(s);
            sp.done.push_back(e);
        }
    }
    *out = &sp;
    return LFRL_OK;
}

// Queue one iteration of the jobs on plan p, in launches of at most
// kMaxBatchJobs frames and the plan's tile capacity.
static int step_plan_group(lfrl_plan_s *p, std::vector<Frame *> &fr, hipStream_t st)
{
    size_t i = 0;
    while (i < fr.size()) {
        int n = 0, tiles = 0;
        while (i + n < fr.size() && n < kMaxBatchJobs) {
            const int t = tiles_for(p->g, fr[i + n]->h, fr[i + n]->w).nt;
            if (n > 0 && tiles + t > p->max_tiles)
                break;
            tiles += t;
            ++n;
        }
        int rc = step_frames(p, fr.data() + i, n, st);
        if (rc)
            return rc;
        for (int k = 0; k < n; ++k)
            if ((rc = frame_queue_poll(*fr[i + k], st)))
                return rc;
        i += n;
    }
    return LFRL_OK;
}

extern "C" int lfrl_job_step(const lfrl_job_t *jobs, int32_t njobs, int32_t *active, void *stream)
{
    if (njobs < 0 || (njobs > 0 && !jobs))
        return set_error(LFRL_ERR_ARG, "bad job list");
    std::vector<lfrl_plan_s *> plans;
    std::vector<std::vector<Frame *>> groups;
    bool any_metric = false;
    int dev = -1;
    for (int i = 0; i < njobs; ++i) {
        if (!jobs[i])
            return set_error(LFRL_ERR_ARG, "job %d is NULL", i);
        lfrl_job_s *j = jobs[i];
        if (dev < 0)
            dev = j->plan->device;
        else if (j->plan->device != dev)
            return set_error(LFRL_ERR_ARG, "jobs on different devices");
        for (int k = 0; k < i; ++k)
            if (jobs[k] == j)
                return set_error(LFRL_ERR_ARG, "job %d listed twice", i);
        if (j->f.done)
            continue;
        size_t g = 0;
        while (g < plans.size() && plans[g] != j->plan)
            ++g;
        if (g == plans.size()) {
            plans.push_back(j->plan);
            groups.emplace_back();
        }
        groups[g].push_back(&j->f);
        any_metric |= j->f.opts.stop == LFRL_STOP_METRIC;
    }
    int rc = LFRL_OK;
    if (!plans.empty()) {
        DevGuard dg(dev);
        hipStream_t st = (hipStream_t)stream;
        if (plans.size() == 1) {
            rc = step_plan_group(plans[0], groups[0], st);
        } else {
            StreamPool *sp = nullptr;
            if ((rc = get_pool(dev, &sp)))
                return rc;
            HIP_TRY(hipEventRecord(sp->fork, st));
            const int nw = (int)std::min<size_t>(plans.size(), sp->s.size());
            for (int w = 0; w < nw; ++w)
                HIP_TRY(hipStreamWaitEvent(sp->s[w], sp->fork, 0));
            for (size_t g = 0; g < plans.size() && rc == LFRL_OK; ++g)
                rc = step_plan_group(plans[g], groups[g], sp->s[g % nw]);
            for (int w = 0; w < nw; ++w) {
                HIP_TRY(hipEventRecord(sp->done[w], sp->s[w]));
                HIP_TRY(hipStreamWaitEvent(st, sp->done[w], 0));
            }
        }
        if (rc)
            return rc;
        // record each stepped job's use on the caller stream, which the worker
        // streams have joined
        for (int i = 0; i < njobs; ++i)
            if ((rc = job_mark(jobs[i], st)))
                return rc;
        if (any_metric)
            HIP_TRY(hipStreamSynchronize(st));
        for (auto &gr : groups)
            for (Frame *f : gr)
                frame_update_done(*f);
    }
    if (active) {
        int n = 0;
        for (int i = 0; i < njobs; ++i)
            n += jobs[i]->f.done ? 0 : 1;
        *active = n;
    }
    return LFRL_OK;
}

extern "C" int lfrl_job_poll(lfrl_job_t j, int32_t *done, int32_t *iters_run)
{
    if (!j)
        return set_error(LFRL_ERR_ARG, "job is NULL");
    if (done)
        *done = j->f.done ? 1 : 0;
    if (iters_run)
        *iters_run = j->f.iters;
    return LFRL_OK;
}

extern "C" int lfrl_job_result(lfrl_job_t j, float *vol, lfrl_rl_report *report, void *stream)
{
    if (!j)
        return set_error(LFRL_ERR_ARG, "job is NULL");
    DevGuard dg(j->plan->device);
    int rc;
    if (vol && (rc = check_buf(vol, (size_t)j->plan->g.Nz * j->f.h * j->f.w * sizeof(float), "vol")))
        return rc;
    if ((rc = frame_result(j->f, j->plan->g.Nz, vol, report, (hipStream_t)stream)))
        return rc;
    return job_mark(j, (hipStream_t)stream);
}

extern "C" int lfrl_job_destroy(lfrl_job_t j)
{
    free_job(j);
    return LFRL_OK;
}

extern "C" int lfrl_deconvolve_batch(const lfrl_plan_t *plans, int32_t n, const int32_t *h,
                                     const int32_t *w, const float *const *imgs,
                                     float *const *vols, const lfrl_rl_opts *opts,
                                     lfrl_rl_report *reports, void *stream)
{
    if (n < 0 || (n > 0 && (!plans || !h || !w || !imgs || !vols || !opts)))
        return set_error(LFRL_ERR_ARG, "NULL argument");
    std::vector<lfrl_job_t> jobs(n, nullptr);
    auto cleanup = [&]() {
        for (lfrl_job_t j : jobs)
            free_job(j);
    };
    int rc = LFRL_OK;
    for (int i = 0; i < n && rc == LFRL_OK; ++i) {
        if (!plans[i] || !vols[i]) {
            rc = set_error(LFRL_ERR_ARG, "frame %d: NULL plan or vol", i);
            break;
        }
        const uint32_t fl = (reports && reports[i].flux_trace) ? LFRL_JOB_FLUX : 0u;
        rc = lfrl_job_create(&jobs[i], plans[i], h[i], w[i], imgs[i],
                             opts[i].init == 1 ? vols[i] : nullptr, &opts[i], fl, stream);
        if (rc == LFRL_OK)
            rc = check_buf(vols[i], (size_t)plans[i]->g.Nz * h[i] * w[i] * sizeof(float), "vol");
    }
    int active = n;
    while (rc == LFRL_OK && active > 0)
        rc = lfrl_job_step(jobs.data(), n, &active, stream);
    for (int i = 0; i < n && rc == LFRL_OK; ++i)
        rc = lfrl_job_result(jobs[i], vols[i], reports ? &reports[i] : nullptr, stream);
    if (rc != LFRL_OK)
        (void)hipStreamSynchronize((hipStream_t)stream);
    cleanup();
    return rc;
}

// Scratch for the plan-less metric entry point: one growable set per device.
// `done` marks the end of the last call's kernels on its stream; the next call
// makes its own stream wait for it, so calls on different streams take turns
// on the shared buffers instead of racing.
struct MetricScratch {
    float *mip = nullptr;
    double *tabH = nullptr, *tabW = nullptr, *T1 = nullptr, *n2p = nullptr, *Fabs = nullptr;
    size_t h_cap = 0, w_cap = 0;
    hipEvent_t done = nullptr;
    bool recorded = false;
};
static std::mutex g_metric_mu;
static std::vector<MetricScratch> g_metric_scratch;

static void free_metric_scratch(MetricScratch &ms)
{
    void *b[] = {ms.mip, ms.tabH, ms.tabW, ms.T1, ms.n2p, ms.Fabs};
    for (void *q : b)
        if (q)
            (void)hipFree(q);
    const hipEvent_t ev = ms.done;
    ms = MetricScratch();
    ms.done = ev;
}

extern "C" int lfrl_metric(int32_t nz, int32_t h, int32_t w, const float *img, double xs,
                           double ys, double *out, void *stream)
{
    return lfrl_metric_ex(nz, h, w, img, xs, ys, LFRL_REGION_TRIANGLE, LFRL_NORM_MATRIX, out,
                          stream);
}

// Argument checks shared by the plan-less metric entry points.
static int check_metric_args(int32_t nz, int32_t h, int32_t w, const float *img, double xs,
                             double ys, int32_t region, int32_t norm, double *out)
{
    if (!img || !out)
        return set_error(LFRL_ERR_ARG, "NULL argument");
    if (nz < 1 || h < 1 || w < 1)
        return set_error(LFRL_ERR_ARG, "nz, h, w must be >= 1");
    if (region < LFRL_REGION_TRIANGLE || region > LFRL_REGION_WHOLE)
        return set_error(LFRL_ERR_ARG, "unknown metric region %d", region);
    if (norm < LFRL_NORM_MATRIX || norm > LFRL_NORM_SPECTRAL)
        return set_error(LFRL_ERR_ARG, "unknown metric norm %d", norm);
    int rc = check_legs(xs, ys, region);
    if (rc || (rc = check_norm_size(norm, h, w)))
        return rc;
    if ((rc = check_buf(img, (size_t)nz * h * w * sizeof(float), "img")) ||
        (rc = check_buf(out, sizeof(double), "out")))
        return rc;
    return LFRL_OK;
}

extern "C" int lfrl_metric_ex(int32_t nz, int32_t h, int32_t w, const float *img, double xs,
                              double ys, int32_t region, int32_t norm, double *out, void *stream)
{
    int rc = check_metric_args(nz, h, w, img, xs, ys, region, norm, out);
    if (rc)
        return rc;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_metric_mu);
    if ((int)g_metric_scratch.size() <= dev)
        g_metric_scratch.resize(dev + 1);
    MetricScratch &ms = g_metric_scratch[dev];
    if (!ms.done)
        HIP_TRY(hipEventCreateWithFlags(&ms.done, hipEventDisableTiming));
    if (ms.h_cap < (size_t)h || ms.w_cap < (size_t)w) {
        if (ms.mip) {
            HIP_TRY(hipDeviceSynchronize());
            free_metric_scratch(ms);
        }
        // room for the whole coefficient matrix of an hc x wc image
        const size_t hc = std::max<size_t>(h, 1024), wc = std::max<size_t>(w, 1024);
        rc = dalloc(&ms.mip, hc * wc * sizeof(float));
        if (!rc) rc = dalloc(&ms.tabH, hc * hc * sizeof(double));
        if (!rc) rc = dalloc(&ms.tabW, wc * wc * sizeof(double));
        if (!rc)
            rc = dalloc(&ms.T1, std::max((size_t)kMetricChunks * kMaxMetricLegs * wc, hc * wc) *
                                    sizeof(double));
        if (!rc) rc = dalloc(&ms.n2p, ((hc * wc + 255) / 256 + 1) * sizeof(double));
        if (!rc) rc = dalloc(&ms.Fabs, hc * wc * sizeof(double));
        if (rc) {
            free_metric_scratch(ms);
            return rc;
        }
        ms.h_cap = hc;
        ms.w_cap = wc;
    }
    const hipStream_t st = (hipStream_t)stream;
    if (ms.recorded)
        HIP_TRY(hipStreamWaitEvent(st, ms.done, 0));
    const MetricBufs mb{ms.mip, ms.tabH, ms.tabW, ms.T1, ms.n2p, ms.Fabs,
                        nullptr, nullptr, nullptr, nullptr};
    rc = run_metric(nz, h, w, img, xs, ys, region, norm, out, mb, nullptr, nullptr, 0, 1, 1, st);
    if (rc)
        return rc;
    HIP_TRY(hipEventRecord(ms.done, st));
    ms.recorded = true;
    return LFRL_OK;
}

// ---------------------------------------------------------------------------
// allocation-free metric: the scratch of lfrl_metric_ex for the triangle and
// rectangle regions in a fixed device array, one copy per GPU, held until the
// process ends.  Layout (byte offsets, each 256-aligned), for images up to
// kStaticSide x kStaticSide and legs up to kMaxMetricLegs bins:
//   mip  [h][w] float                          4 MiB
//   tabH [nv][h], tabW [nu][w] double          2 + 2 MiB
//   T1   [nchunks][nv][w] double, nchunks * nv <= kMetricChunks * kMaxMetricLegs
//        (also the entropy partials of large coefficient sets)  16 MiB
//   n2p  [(h w + 255) / 256 + 1] double         32 KiB
//   Fabs [nv][nu] double                        512 KiB
static constexpr int kStaticSide = 1024;
static constexpr size_t kStaticMip = 0;
static constexpr size_t kStaticTabH = kStaticMip + (size_t)kStaticSide * kStaticSide * sizeof(float);
static constexpr size_t kStaticTabW =
    kStaticTabH + (size_t)kMaxMetricLegs * kStaticSide * sizeof(double);
static constexpr size_t kStaticT1 =
    kStaticTabW + (size_t)kMaxMetricLegs * kStaticSide * sizeof(double);
static constexpr size_t kStaticN2p =
    kStaticT1 + (size_t)kMetricChunks * kMaxMetricLegs * kStaticSide * sizeof(double);
static constexpr size_t kStaticFabs =
    kStaticN2p + (((size_t)kStaticSide * kStaticSide + 255) / 256 + 1 + 31) / 32 * 32 * sizeof(double);
static constexpr size_t kStaticBytes =
    kStaticFabs + (size_t)kMaxMetricLegs * kMaxMetricLegs * sizeof(double);
static_assert(kStaticTabH % 256 == 0 && kStaticTabW % 256 == 0 && kStaticT1 % 256 == 0 &&
                  kStaticN2p % 256 == 0 && kStaticFabs % 256 == 0,
              "static metric scratch offsets must stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// Device address of `scratch` on each GPU, looked up once per device with that
// device current (the host-side name is only a stand-in for the symbol).
static constexpr int kStaticMaxDevices = 64;
static std::mutex g_static_mu;
static unsigned char *g_static_ptr[kStaticMaxDevices] = {};

static int static_scratch(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kStaticMaxDevices)
        return set_error(LFRL_ERR_UNSUPPORTED, "device %d beyond %d", dev, kStaticMaxDevices);
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p)
            return set_error(LFRL_ERR_DEVICE, "no device address for the metric scratch");
        g_static_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_static_ptr[dev];
    return LFRL_OK;
}

extern "C" int lfrl_metric_noalloc(int32_t nz, int32_t h, int32_t w, const float *img, double xs,
                                   double ys, int32_t region, int32_t norm, double *out,
                                   void *stream)
{
    int rc = check_metric_args(nz, h, w, img, xs, ys, region, norm, out);
    if (rc)
        return rc;
    if (region == LFRL_REGION_WHOLE)
        return set_error(LFRL_ERR_UNSUPPORTED,
                         "lfrl_metric_noalloc serves the triangle and rectangle regions only");
    if (h > kStaticSide || w > kStaticSide)
        return set_error(LFRL_ERR_UNSUPPORTED,
                         "lfrl_metric_noalloc serves images up to %d x %d (got %d x %d)",
                         kStaticSide, kStaticSide, h, w);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    unsigned char *base = nullptr;
    if ((rc = static_scratch(dev, &base)))
        return rc;
    const MetricBufs mb{reinterpret_cast<float *>(base + kStaticMip),
                        reinterpret_cast<double *>(base + kStaticTabH),
                        reinterpret_cast<double *>(base + kStaticTabW),
                        reinterpret_cast<double *>(base + kStaticT1),
                        reinterpret_cast<double *>(base + kStaticN2p),
                        reinterpret_cast<double *>(base + kStaticFabs),
                        nullptr, nullptr, nullptr, nullptr};
    return run_metric(nz, h, w, img, xs, ys, region, norm, out, mb, nullptr, nullptr, 0, 1, 1,
                      (hipStream_t)stream);
}

extern "C" int lfrl_metric_cutoff(double d_ml, double mag, int32_t nnum, double lambda, double na,
                                  int32_t h, int32_t w, double *xs, double *ys)
{
    if (!xs || !ys)
        return set_error(LFRL_ERR_ARG, "NULL argument");
    if (!(d_ml > 0) || !(mag > 0) || nnum < 1 || !(lambda > 0) || !(na > 0) || h < 1 || w < 1)
        return set_error(LFRL_ERR_ARG, "optics parameters must be positive");
    const double pu = d_ml / (mag * nnum);
    const double dpsf = 1.22 * lambda * nnum / na;
    *xs = pu * w / dpsf;
    *ys = pu * h / dpsf;
    return LFRL_OK;
}

extern "C" int lfrl_profile_enable(lfrl_plan_t p, int32_t on)
{
    if (!p)
        return set_error(LFRL_ERR_ARG, "NULL plan");
    p->prof = on != 0;
    p->ev_used[0] = p->ev_used[1] = 0;
    return LFRL_OK;
}

extern "C" int lfrl_profile_read(lfrl_plan_t p, const char *kernel, double *total_ms,
                                 int64_t *launches)
{
    if (!p || !kernel || !total_ms || !launches)
        return set_error(LFRL_ERR_ARG, "NULL argument");
    int which = -1;
    if (!strcmp(kernel, "contract_fwd"))
        which = 0;
    else if (!strcmp(kernel, "contract_adj"))
        which = 1;
    if (which < 0)
        return set_error(LFRL_ERR_ARG, "unknown kernel '%s'", kernel);
    DevGuard dg(p->device);
    double tot = 0.0;
    const size_t used = p->ev_used[which];
    for (size_t i = 0; i + 1 < used; i += 2) {
        HIP_TRY(hipEventSynchronize(p->ev[which][i + 1]));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p->ev[which][i], p->ev[which][i + 1]));
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)(used / 2);
    return LFRL_OK;
}

// ---------------------------------------------------------------------------
// PSF from optical parameters (sec. 2.1, Fig. 1)
#include "psf_optics.hpp"

// Gauss-Legendre nodes and weights on [lo, hi]: Newton's method on P_n (three-
// term recurrence), started from the usual cosine estimates of its roots.
static void gauss_legendre(int n, double lo, double hi, std::vector<double> &x,
                           std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double mid = 0.5 * (hi + lo), half = 0.5 * (hi - lo);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;   // P_0, P_1
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_n(z), p0 = P_{n-1}(z)
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16)
                break;
        }
        const double wt = 2.0 / ((1.0 - z * z) * dp * dp);
        x[i] = mid - half * z;          // ascending order
        x[n - 1 - i] = mid + half * z;
        w[i] = w[n - 1 - i] = half * wt;
    }
}

static int nice_fft_size(int n)
{
    for (int m = std::max(1, n);; ++m) {
        int q = m;
        for (int p : {2, 3, 5})
            while (q % p == 0)
                q /= p;
        if (q == 1)
            return m;
    }
}

static bool fft_plan_for(int n, psfopt::FftPlan *plan)
{
    plan->n = n;
    plan->nst = 0;
    int q = n;
    for (int r : {4, 2, 3, 5})
        while (q % r == 0) {
            if (plan->nst == psfopt::kMaxStages)
                return false;
            plan->radix[plan->nst++] = r;
            q /= r;
        }
    return q == 1;
}

// Device buffers of one PSF computation.
struct PsfScratch {
    double2 *e = nullptr, *U = nullptr;
    double *s = nullptr;
    float2 *tw = nullptr, *hx = nullptr, *W = nullptr;
    ~PsfScratch()
    {
        void *b[] = {e, U, s, tw, hx, W};
        for (void *p : b)
            if (p)
                (void)hipFree(p);
    }
};

static constexpr size_t kPsfWorkBytes = (size_t)1 << 30;  // field batch buffer

static int check_optics(const lfrl_optics *o, const double *depths)
{
    if (!o || !depths)
        return set_error(LFRL_ERR_ARG, "NULL argument");
    const double v[] = {o->wavelength, o->na, o->n_medium, o->mag, o->d_ml, o->f_ml};
    for (double x : v)
        if (!(x > 0.0) || !std::isfinite(x))
            return set_error(LFRL_ERR_ARG, "optical parameters must be positive and finite");
    if (!(o->na < o->n_medium))
        return set_error(LFRL_ERR_ARG, "NA %g must be below the medium index %g", o->na,
                         o->n_medium);
    if (o->nnum < 1 || o->nnum > 64 || o->nz < 1 || o->ksize < 1 || o->ksize % 2 == 0 ||
        o->osr < 1 || o->osr % 2 == 0 || o->nquad < 0 || o->nquad > 65536)
        return set_error(LFRL_ERR_ARG,
                         "need 1 <= nnum <= 64, nz >= 1, odd ksize and osr, 0 <= nquad <= 65536");
    for (int j = 0; j < o->nz; ++j)
        if (!std::isfinite(depths[j]))
            return set_error(LFRL_ERR_ARG, "depth %d is not finite", j);
    return LFRL_OK;
}

extern "C" int lfrl_psf_compute(const lfrl_optics *o, const double *depths, float *psf,
                                void *stream)
{
    int rc = check_optics(o, depths);
    if (rc)
        return rc;
    using namespace psfopt;
    const int N = o->nnum, K = o->ksize, osr = o->osr, nz = o->nz;
    const int nq = o->nquad ? o->nquad : 1024;
    if ((long long)K * osr > kMaxSide)
        return set_error(LFRL_ERR_UNSUPPORTED, "ksize * osr = %lld above %d samples",
                         (long long)K * osr, kMaxSide);
    Window w;
    w.K = K;
    w.osr = osr;
    w.N = N;
    w.G = K * osr;
    w.Gf = nice_fft_size(w.G);
    if (w.Gf > kMaxSide)
        return set_error(LFRL_ERR_UNSUPPORTED, "FFT grid %d above %d", w.Gf, kMaxSide);
    w.off = (w.Gf - w.G) / 2;
    w.hh = (w.G - 1) / 2;
    w.pixel = o->d_ml / N;
    w.lens_k = M_PI / (o->wavelength * o->f_ml);
    const int n = w.Gf;
    FftPlan plan;
    if (!fft_plan_for(n, &plan))
        return set_error(LFRL_ERR_UNSUPPORTED, "FFT size %d", n);
    const size_t nfield = (size_t)N * N;
    if ((rc = check_buf(psf, (size_t)nz * nfield * K * K * sizeof(float), "psf")))
        return rc;
    const hipStream_t st = (hipStream_t)stream;
    const double delta = w.pixel / osr;

    // quadrature coefficients: e[j][q] = w_q sqrt(cos t) sin t exp(i k n z_j (1 - cos t)),
    // s[q] = k n sin t / M (J0 argument per unit image radius)
    const double alpha = std::asin(o->na / o->n_medium);
    const double kn = 2.0 * M_PI / o->wavelength * o->n_medium;
    std::vector<double> t, wq;
    gauss_legendre(nq, 0.0, alpha, t, wq);
    std::vector<double2> e((size_t)nz * nq);
    std::vector<double> s(nq);
    for (int q = 0; q < nq; ++q)
        s[q] = kn * std::sin(t[q]) / o->mag;
    for (int j = 0; j < nz; ++j)
        for (int q = 0; q < nq; ++q) {
            const double amp = wq[q] * std::sqrt(std::cos(t[q])) * std::sin(t[q]);
            const double ph = kn * depths[j] * (1.0 - std::cos(t[q]));
            e[(size_t)j * nq + q] = make_double2(amp * std::cos(ph), amp * std::sin(ph));
        }
    // DFT roots and the 1-D factor of the transfer function
    std::vector<float2> tw(n), hx(n);
    for (int m = 0; m < n; ++m) {
        const double a = 2.0 * M_PI * m / n;
        tw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
        const int kf = 2 * m < n ? m : m - n;
        const double fk = kf / (n * delta);
        const double ph = -M_PI * o->wavelength * o->f_ml * fk * fk;
        hx[m] = make_float2((float)std::cos(ph), (float)std::sin(ph));
    }
    const int nrad = (w.hh + 1) * (w.hh + 2) / 2;
    const size_t field_bytes = (size_t)w.G * n * sizeof(float2);
    int nb = (int)std::max<size_t>(1, std::min(nfield, kPsfWorkBytes / field_bytes));
    if (const char *cap = std::getenv("LFRL_PSF_BATCH"))   // test hook: smaller field batches
        nb = std::max(1, std::min(nb, std::atoi(cap)));

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    PsfScratch sc;
    if ((rc = dalloc(&sc.e, e.size() * sizeof(double2))) ||
        (rc = dalloc(&sc.s, s.size() * sizeof(double))) ||
        (rc = dalloc(&sc.U, (size_t)nz * nrad * sizeof(double2))) ||
        (rc = dalloc(&sc.tw, n * sizeof(float2))) || (rc = dalloc(&sc.hx, n * sizeof(float2))) ||
        (rc = dalloc(&sc.W, (size_t)nb * field_bytes)))
        return rc;
    HIP_TRY(hipMemcpyAsync(sc.e, e.data(), e.size() * sizeof(double2), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(sc.s, s.data(), s.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(sc.tw, tw.data(), n * sizeof(float2), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(sc.hx, hx.data(), n * sizeof(float2), hipMemcpyHostToDevice, st));

    hipLaunchKernelGGL(k_debye, dim3((nrad + kThreads - 1) / kThreads,
                                     (nz + kDepthsPerThread - 1) / kDepthsPerThread),
                       dim3(kThreads), 0, st, (const double2 *)sc.e, (const double *)sc.s, nq, nz,
                       nrad, delta, sc.U);
    LAUNCH_CHECK("k_debye");

    const int lines = std::max(1, kLineBudget / n);
    const int nl_rows = lines, S = lines, nl_bin = std::min(osr, lines);
    const size_t lds_rows = ((size_t)n + w.G + (size_t)nl_rows * n) * sizeof(float2);
    const size_t lds_cols = ((size_t)n + (size_t)S * n) * sizeof(float2);
    const size_t lds_bin = ((size_t)n + (w.G + 1) / 2 + (size_t)nl_bin * n) * sizeof(float2);
    raise_lds_attr((const void *)k_psf_rows, lds_rows);
    raise_lds_attr((const void *)k_psf_cols, lds_cols);
    raise_lds_attr((const void *)k_psf_bin, lds_bin);
    for (int j = 0; j < nz; ++j) {
        const double2 *Uj = sc.U + (size_t)j * nrad;
        float *psf_j = psf + (size_t)j * nfield * K * K;
        for (int f0 = 0; f0 < (int)nfield; f0 += nb) {
            const int nf = std::min(nb, (int)nfield - f0);
            hipLaunchKernelGGL(k_psf_rows, dim3((w.G + nl_rows - 1) / nl_rows, nf), dim3(kThreads),
                               lds_rows, st, Uj, nrad, w, plan, (const float2 *)sc.tw, nl_rows, f0,
                               sc.W);
            LAUNCH_CHECK("k_psf_rows");
            hipLaunchKernelGGL(k_psf_cols, dim3((n + S - 1) / S, nf), dim3(kThreads), lds_cols, st,
                               w, plan, (const float2 *)sc.tw, (const float2 *)sc.hx, S, sc.W);
            LAUNCH_CHECK("k_psf_cols");
            hipLaunchKernelGGL(k_psf_bin, dim3(K, nf), dim3(kThreads), lds_bin, st, w, plan,
                               (const float2 *)sc.tw, nl_bin, (const float2 *)sc.W, f0, psf_j);
            LAUNCH_CHECK("k_psf_bin");
        }
    }
    if (o->flags & LFRL_PSF_UNIT_SUM) {
        hipLaunchKernelGGL(k_normalize_psf, dim3((unsigned)(nz * nfield)), dim3(256), 0, st, psf,
                           (size_t)K * K);
        LAUNCH_CHECK("k_normalize_psf");
    }
    HIP_TRY(hipStreamSynchronize(st));
    return LFRL_OK;
}

extern "C" const char *lfrl_last_error(void)
{
    return g_last_error.c_str();
}
