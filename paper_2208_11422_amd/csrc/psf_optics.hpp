// psf_optics.hpp - the light-field PSF computed on the GPU from optical
// parameters (sec. 2.1: the PSF computation moved to the GPU; Fig. 1: computed
// from the system's parameters is the default PSF source).  Included by
// lfrl.hip.
//
// Model (scalar wave optics of the light-field microscope):
//   1. native-image-plane field of an on-axis point source at depth z, from the
//      Debye integral of a sine-condition objective,
//        U(r, z) = int_0^alpha sqrt(cos t) sin t exp(i k n z (1 - cos t))
//                               J0(k n r sin t / M) dt,   alpha = asin(NA / n),
//      by Gauss-Legendre quadrature (constant factors and the depth-only phase
//      dropped);
//   2. the thin-lens phase exp(-i pi |x - c|^2 / (lambda f_ml)) of every
//      lenslet about its centre c;
//   3. Fresnel propagation over f_ml with the transfer function
//      exp(-i pi lambda f_ml (fx^2 + fy^2)) on a periodic Gf x Gf grid;
//   4. |U|^2 summed over the osr x osr samples of every pixel.
// Grid: pixel pitch p = d_ml / nnum, sample spacing p / osr, a window of
// K x K pixels (G = K osr samples) centred on the source pixel, placed at
// offset (Gf - G) / 2 of the FFT grid, zero outside.
//
// GPU layout of the work:
//   k_debye        U[j][rho] for every distinct window radius (rho indexes
//                  0 <= n <= m <= (G - 1) / 2 as m (m + 1) / 2 + n), float64:
//                  the quadrature is a sum of ~1000 oscillating terms whose
//                  result can be far smaller than its terms (diffraction
//                  tails), so it is summed in float64 (a small, once-per-set
//                  cost); one thread per radius, 8 depths per thread.
//   k_psf_rows     window rows of one source's lenslet-array field, forward
//                  row DFTs in LDS, written to the work buffer (float32).
//   k_psf_cols     columns: forward DFT, transfer function, inverse DFT, in LDS.
//   k_psf_bin      inverse row DFTs of the window rows, |U|^2, pixel sums.
// The DFTs are in-place Stockham passes over lines held in LDS, each thread
// holding its butterflies' inputs in registers between two barriers.
#pragma once

namespace psfopt {

static constexpr int kMaxStages = 16;
static constexpr int kMaxSide = 2048;   // largest FFT grid side
static constexpr int kThreads = 512;
static constexpr int kLineBudget = 15 * kThreads;  // complex values a block transforms at once
static constexpr int kDepthsPerThread = 8;
static constexpr int kQuadChunk = 256;

struct FftPlan {
    int n;
    int nst;
    int radix[kMaxStages];
};

// One radix-R Stockham stage over nl lines of length n held in buf, in place:
// every thread loads the inputs of its butterflies into registers, the block
// synchronises, then every thread writes its outputs.
template <int R, int SIGN>
__device__ __forceinline__ void lds_stage(float2 *buf, int nl, int n, int ns,
                                          const float2 *__restrict__ tw)
{
    constexpr int kMaxB = (kLineBudget / kThreads + R - 1) / R;  // butterflies per thread
    const int per = n / R;
    const int nb = nl * per;
    const int tstep = n / (ns * R);
    float2 v[kMaxB][R];
#pragma unroll
    for (int i = 0; i < kMaxB; ++i) {
        const int bf = threadIdx.x + i * kThreads;
        if (bf < nb) {
            const int line = bf / per, idx = bf % per;
            const int k = idx % ns;
            const float2 *src = buf + (size_t)line * n + idx;
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[i][r] = src[r * per];
            if (k != 0) {
#pragma unroll
                for (int r = 1; r < R; ++r)
                    v[i][r] = tfft::cmulf(v[i][r], tfft::twid<SIGN>(tw, (k * r * tstep) % n));
            }
            tfft::dft_small<R, SIGN, 1>(v[i], tw);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kMaxB; ++i) {
        const int bf = threadIdx.x + i * kThreads;
        if (bf < nb) {
            const int line = bf / per, idx = bf % per;
            const int k = idx % ns;
            float2 *dst = buf + (size_t)line * n + (idx / ns) * ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r)
                dst[r * ns] = v[i][r];
        }
    }
    __syncthreads();
}

// nl unnormalised DFTs of length plan.n over contiguous lines of buf:
// X[k] = sum_m x[m] exp(SIGN 2 pi i k m / n).  tw[m] = exp(2 pi i m / n).
// Requires nl * n <= kLineBudget and a barrier before (the lines written).
template <int SIGN>
__device__ void lds_fft(float2 *buf, int nl, const FftPlan &plan, const float2 *__restrict__ tw)
{
    int ns = 1;
    for (int s = 0; s < plan.nst; ++s) {
        const int r = plan.radix[s];
        if (r == 4)
            lds_stage<4, SIGN>(buf, nl, plan.n, ns, tw);
        else if (r == 2)
            lds_stage<2, SIGN>(buf, nl, plan.n, ns, tw);
        else if (r == 3)
            lds_stage<3, SIGN>(buf, nl, plan.n, ns, tw);
        else
            lds_stage<5, SIGN>(buf, nl, plan.n, ns, tw);
        ns *= r;
    }
}

// Window geometry shared by the three field kernels.
struct Window {
    int G, Gf, off, hh;   // samples per side, FFT side, window offset, (G - 1) / 2
    int K, osr, N;        // pixels per side, samples per pixel, pixels per lenslet
    double pixel;         // pixel pitch
    double lens_k;        // pi / (lambda f_ml)
};

// Distinct-radius index of window offsets (m, n).
__device__ __forceinline__ int radius_index(int m, int n)
{
    m = abs(m);
    n = abs(n);
    const int hi = max(m, n), lo = min(m, n);
    return hi * (hi + 1) / 2 + lo;
}

// Pixel offset from a window sample (idx samples from the source pixel centre)
// to the centre of the lenslet it lies under, for a source of phase `phase`.
__device__ __forceinline__ double lens_offset(int idx, int phase, const Window &w)
{
    const double pix = (double)idx / w.osr;
    const double lens = floor((pix + phase + 0.5) / w.N);
    const double centre = w.N * lens + 0.5 * (w.N - 1) - phase;
    return pix - centre;
}

// U[j][rho] = sum_q e[j][q] J0(s[q] r_rho), r_rho = delta sqrt(m^2 + n^2).
// Grid: (ceil(nrad / kThreads), ceil(nz / kDepthsPerThread)).
__global__ __launch_bounds__(kThreads) void k_debye(const double2 *__restrict__ e,
                                                    const double *__restrict__ s, int nq, int nz,
                                                    int nrad, double delta,
                                                    double2 *__restrict__ U)
{
    __shared__ double2 es[kDepthsPerThread][kQuadChunk];
    __shared__ double ss[kQuadChunk];
    const int rho = blockIdx.x * kThreads + threadIdx.x;
    const int jz = blockIdx.y * kDepthsPerThread;
    const int nd = min(kDepthsPerThread, nz - jz);
    // (m, n) from rho = m (m + 1) / 2 + n, 0 <= n <= m
    int m = (int)floor((sqrt(8.0 * (double)rho + 1.0) - 1.0) * 0.5);
    while (m * (m + 1) / 2 > rho)
        --m;
    while ((m + 1) * (m + 2) / 2 <= rho)
        ++m;
    const int nn = rho - m * (m + 1) / 2;
    const double r = delta * sqrt((double)m * m + (double)nn * nn);
    double2 acc[kDepthsPerThread];
#pragma unroll
    for (int d = 0; d < kDepthsPerThread; ++d)
        acc[d] = make_double2(0.0, 0.0);
    for (int q0 = 0; q0 < nq; q0 += kQuadChunk) {
        const int nc = min(kQuadChunk, nq - q0);
        __syncthreads();
        for (int i = threadIdx.x; i < kDepthsPerThread * kQuadChunk; i += kThreads) {
            const int d = i / kQuadChunk, q = i % kQuadChunk;
            es[d][q] = (d < nd && q < nc) ? e[(size_t)(jz + d) * nq + q0 + q]
                                          : make_double2(0.0, 0.0);
        }
        for (int q = threadIdx.x; q < kQuadChunk; q += kThreads)
            ss[q] = q < nc ? s[q0 + q] : 0.0;
        __syncthreads();
        if (rho < nrad) {
            for (int q = 0; q < nc; ++q) {
                const double jv = j0(ss[q] * r);
#pragma unroll
                for (int d = 0; d < kDepthsPerThread; ++d) {
                    acc[d].x = fma(es[d][q].x, jv, acc[d].x);
                    acc[d].y = fma(es[d][q].y, jv, acc[d].y);
                }
            }
        }
    }
    if (rho < nrad) {
#pragma unroll
        for (int d = 0; d < kDepthsPerThread; ++d)
            if (d < nd)
                U[(size_t)(jz + d) * nrad + rho] = acc[d];
    }
}

// Field on nl window rows of one source (the depth's Debye field times the
// lenslet phases), forward DFT along each row, stored as window rows of the
// work buffer W[field][G][Gf].  Grid: (ceil(G / nl), fields); field f of the
// launch is source phase (a, b) = ((f0 + f) / N, (f0 + f) % N).
__global__ __launch_bounds__(kThreads) void k_psf_rows(const double2 *__restrict__ Uj, int nrad,
                                                       const Window w, const FftPlan plan,
                                                       const float2 *__restrict__ twg, int nl,
                                                       int f0, float2 *__restrict__ W)
{
    extern __shared__ float2 lds[];
    const int n = w.Gf;
    float2 *tw = lds;
    float2 *colf = tw + n;        // [G] column lenslet phases
    float2 *buf = colf + w.G;     // [nl][n]
    const int f = f0 + blockIdx.y, a = f / w.N, b = f % w.N;
    const int row0 = blockIdx.x * nl;
    for (int i = threadIdx.x; i < n; i += kThreads)
        tw[i] = twg[i];
    for (int c = threadIdx.x; c < w.G; c += kThreads) {
        const double dx = lens_offset(c - w.hh, b, w) * w.pixel;
        double sn, cs;
        sincos(-w.lens_k * dx * dx, &sn, &cs);
        colf[c] = make_float2((float)cs, (float)sn);
    }
    __syncthreads();
    for (int line = 0; line < nl; ++line) {
        const int wr = row0 + line;
        if (wr >= w.G)
            break;
        const int m = wr - w.hh;
        const double dy = lens_offset(m, a, w) * w.pixel;
        double sn, cs;
        sincos(-w.lens_k * dy * dy, &sn, &cs);
        for (int c = threadIdx.x; c < n; c += kThreads) {
            const int wc = c - w.off;
            float2 v = make_float2(0.f, 0.f);
            if (wc >= 0 && wc < w.G) {
                const double2 u = Uj[radius_index(m, wc - w.hh)];
                // u * row phase in float64, then the column phase in float32
                const float2 ur = make_float2((float)(u.x * cs - u.y * sn),
                                              (float)(u.x * sn + u.y * cs));
                v = tfft::cmulf(ur, colf[wc]);
            }
            buf[(size_t)line * n + c] = v;
        }
    }
    const int rows = min(nl, w.G - row0);
    __syncthreads();
    lds_fft<-1>(buf, rows, plan, tw);
    float2 *dst = W + ((size_t)blockIdx.y * w.G + row0) * n;
    for (int i = threadIdx.x; i < rows * n; i += kThreads)
        dst[i] = buf[i];
}

// Columns c0 .. c0 + S - 1 of one field: rows outside the window are zero;
// forward DFT along the column, times the transfer function
// hx[kr] * hx[kc], inverse DFT, window rows written back.  LDS holds the
// strip transposed (one line per column).  Grid: (ceil(Gf / S), fields).
__global__ __launch_bounds__(kThreads) void k_psf_cols(const Window w, const FftPlan plan,
                                                       const float2 *__restrict__ twg,
                                                       const float2 *__restrict__ hx, int S,
                                                       float2 *__restrict__ W)
{
    extern __shared__ float2 lds[];
    const int n = w.Gf;
    float2 *tw = lds;
    float2 *buf = tw + n;   // [S][n]
    const int c0 = blockIdx.x * S;
    const int cols = min(S, n - c0);
    float2 *fld = W + (size_t)blockIdx.y * w.G * n;
    for (int i = threadIdx.x; i < n; i += kThreads)
        tw[i] = twg[i];
    for (int i = threadIdx.x; i < S * n; i += kThreads) {
        const int r = i / S, cc = i % S;   // cc fastest: contiguous global reads
        const int wr = r - w.off;
        float2 v = make_float2(0.f, 0.f);
        if (cc < cols && wr >= 0 && wr < w.G)
            v = fld[(size_t)wr * n + c0 + cc];
        buf[(size_t)cc * n + r] = v;
    }
    __syncthreads();
    lds_fft<-1>(buf, cols, plan, tw);
    for (int i = threadIdx.x; i < cols * n; i += kThreads) {
        const int cc = i / n, kr = i % n;
        buf[i] = tfft::cmulf(buf[i], tfft::cmulf(hx[kr], hx[c0 + cc]));
    }
    __syncthreads();
    lds_fft<1>(buf, cols, plan, tw);
    for (int i = threadIdx.x; i < S * n; i += kThreads) {
        const int r = i / S, cc = i % S;
        const int wr = r - w.off;
        if (cc < cols && wr >= 0 && wr < w.G)
            fld[(size_t)wr * n + c0 + cc] = buf[(size_t)cc * n + r];
    }
}

// Pixel row u of one field: inverse DFT of its osr window rows (in groups of
// nl rows), |U|^2 / Gf^4, summed over each pixel's osr x osr samples, written
// to psf[j][a][b][u][0..K).  Grid: (K, fields).
__global__ __launch_bounds__(kThreads) void k_psf_bin(const Window w, const FftPlan plan,
                                                      const float2 *__restrict__ twg, int nl,
                                                      const float2 *__restrict__ W, int f0,
                                                      float *__restrict__ psf_j)
{
    extern __shared__ float2 lds[];
    const int n = w.Gf;
    float2 *tw = lds;
    float *acc = reinterpret_cast<float *>(tw + n);            // [G]
    float2 *buf = tw + n + (w.G + 1) / 2;                      // [nl][n]
    const int u = blockIdx.x;
    const float2 *fld = W + (size_t)blockIdx.y * w.G * n;
    const float scale = 1.0f / ((float)n * (float)n);
    for (int i = threadIdx.x; i < n; i += kThreads)
        tw[i] = twg[i];
    for (int i = threadIdx.x; i < w.G; i += kThreads)
        acc[i] = 0.f;
    for (int t0 = 0; t0 < w.osr; t0 += nl) {
        const int rows = min(nl, w.osr - t0);
        __syncthreads();
        for (int i = threadIdx.x; i < rows * n; i += kThreads)
            buf[i] = fld[(size_t)(u * w.osr + t0) * n + i];
        __syncthreads();
        lds_fft<1>(buf, rows, plan, tw);
        for (int c = threadIdx.x; c < w.G; c += kThreads) {
            float s = acc[c];
            for (int r = 0; r < rows; ++r) {
                const float2 v = buf[(size_t)r * n + w.off + c];
                const float re = v.x * scale, im = v.y * scale;
                s += re * re + im * im;
            }
            acc[c] = s;
        }
    }
    __syncthreads();
    const int f = f0 + blockIdx.y;
    float *out = psf_j + (size_t)f * w.K * w.K + (size_t)u * w.K;
    for (int v = threadIdx.x; v < w.K; v += kThreads) {
        float s = 0.f;
        for (int t = 0; t < w.osr; ++t)
            s += acc[v * w.osr + t];
        out[v] = s;
    }
}

}  // namespace psfopt
