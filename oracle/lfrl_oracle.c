/*
 * CPU reference ("oracle") for light-field Richardson-Lucy deconvolution.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liblfrl_oracle.so, which
 * only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * load.  It shares no code with the HIP library and never sees its outputs.
 *
 * Plain, slow, obviously correct: direct spatial loops in float64, no FFT, no
 * tiling, no reordering beyond what the definitions state.  The PSF arrives as
 * the same float32 taps the GPU gets and each tap is promoted to float64 where
 * it is used.
 *
 * Definitions (the paper, sec. 1, names 3-D Richardson-Lucy deconvolution of the
 * light-field image following Prevedel et al. 2014; the light-field forward model
 * is a per-depth, per-lenslet-phase convolution):
 *
 *   PSF      h[j][a][b][u][v]: image of a point source in depth plane j whose
 *            pixel has row phase a = r mod N and column phase b = s mod N, tap
 *            (u, v) sitting at displacement (u - c0, v - c0), c0 = (K - 1) / 2.
 *   forward  y[pr][ps] = sum_j sum_{r,s} x[j][r][s] *
 *                        h[j][r mod N][s mod N][pr - r + c0][ps - s + c0]
 *            (taps outside [0, K) are zero; pixels outside the image are zero:
 *            linear, zero-padded, "same"-size projection).
 *   backward the exact adjoint of forward:
 *            b[j][r][s] = sum_{pr,ps} y[pr][ps] *
 *                         h[j][r mod N][s mod N][pr - r + c0][ps - s + c0].
 *
 * Parity is pinned by the tests (delta voxel, Nnum = 1 against a library 2-D
 * convolution, adjointness, superposition), not by this file itself.
 */
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline size_t psf_index(int nnum, int ksize, int j, int a, int b)
{
    return ((((size_t)j * nnum + a) * nnum + b) * ksize) * ksize;
}

/* Forward projection, written as the superposition of point images: every
 * voxel adds its PSF, weighted by its value, centred on its own pixel.  Voxels
 * that are exactly zero add nothing and are skipped.  Rows of the volume are
 * split statically over threads; each thread accumulates into its own image and
 * the images are summed in thread order, so a fixed thread count gives a
 * bit-identical result. */
int oracle_forward(int nnum, int nz, int ksize, int h, int w,
                   const float *psf, const double *vol, double *img)
{
    if (nnum < 1 || nz < 1 || ksize < 1 || (ksize & 1) == 0 || h < 0 || w < 0)
        return -1;
    const int c0 = (ksize - 1) / 2;
    const size_t npx = (size_t)h * w;
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double *acc = (double *)calloc((size_t)nthreads * (npx ? npx : 1), sizeof(double));
    if (!acc)
        return -2;
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = acc + (size_t)tid * npx;
        long rows = (long)nz * h;
#pragma omp for schedule(static)
        for (long jr = 0; jr < rows; ++jr) {
            const int j = (int)(jr / h), r = (int)(jr % h);
            for (int s = 0; s < w; ++s) {
                const double xv = vol[((size_t)j * h + r) * w + s];
                if (xv == 0.0)
                    continue;
                const float *k = psf + psf_index(nnum, ksize, j, r % nnum, s % nnum);
                for (int u = 0; u < ksize; ++u) {
                    const int pr = r + u - c0;
                    if (pr < 0 || pr >= h)
                        continue;
                    for (int v = 0; v < ksize; ++v) {
                        const int ps = s + v - c0;
                        if (ps < 0 || ps >= w)
                            continue;
                        mine[(size_t)pr * w + ps] += xv * (double)k[(size_t)u * ksize + v];
                    }
                }
            }
        }
    }
    memset(img, 0, npx * sizeof(double));
    for (int t = 0; t < nthreads; ++t)
        for (size_t i = 0; i < npx; ++i)
            img[i] += acc[(size_t)t * npx + i];
    free(acc);
    return 0;
}

/* One forward-projected pixel, written as the gather over every voxel whose PSF
 * reaches it (the same sum as oracle_forward, evaluated at one output). */
static double forward_pixel(int nnum, int nz, int ksize, int h, int w,
                            const float *psf, const double *vol, int pr, int ps)
{
    const int c0 = (ksize - 1) / 2;
    double sum = 0.0;
    for (int j = 0; j < nz; ++j) {
        for (int u = 0; u < ksize; ++u) {
            const int r = pr - u + c0;
            if (r < 0 || r >= h)
                continue;
            for (int v = 0; v < ksize; ++v) {
                const int s = ps - v + c0;
                if (s < 0 || s >= w)
                    continue;
                const float *k = psf + psf_index(nnum, ksize, j, r % nnum, s % nnum);
                sum += vol[((size_t)j * h + r) * w + s] * (double)k[(size_t)u * ksize + v];
            }
        }
    }
    return sum;
}

/* Forward projection evaluated only at the listed pixels (pr[i], ps[i]). */
int oracle_forward_at(int nnum, int nz, int ksize, int h, int w,
                      const float *psf, const double *vol,
                      long npts, const int *pr, const int *ps, double *out)
{
    if (nnum < 1 || nz < 1 || ksize < 1 || (ksize & 1) == 0)
        return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (long i = 0; i < npts; ++i)
        out[i] = forward_pixel(nnum, nz, ksize, h, w, psf, vol, pr[i], ps[i]);
    return 0;
}

/* Forward projection evaluated on the pixel window rows [r0, r1) x columns
 * [s0, s1) (clipped to the image), out[(pr - r0) * (s1 - s0) + (ps - s0)].  The
 * same sum as oracle_forward restricted to those outputs, gathered one output
 * row at a time: for output row pr, every voxel row r whose PSF tap row
 * u = pr - r + c0 lies in [0, K) adds its taps along that row.  Each output row
 * is summed by one thread in the order (j, r, s, v), so the values do not
 * depend on the thread count.  Pixels of the window outside the image are 0. */
int oracle_forward_window(int nnum, int nz, int ksize, int h, int w,
                          const float *psf, const double *vol,
                          int r0, int r1, int s0, int s1, double *out)
{
    if (nnum < 1 || nz < 1 || ksize < 1 || (ksize & 1) == 0 || r1 < r0 || s1 < s0)
        return -1;
    const int c0 = (ksize - 1) / 2;
    const int ww = s1 - s0;
    memset(out, 0, (size_t)(r1 - r0) * (size_t)ww * sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int pr = r0; pr < r1; ++pr) {
        if (pr < 0 || pr >= h)
            continue;
        double *orow = out + (size_t)(pr - r0) * ww;
        const int pc0 = s0 > 0 ? s0 : 0, pc1 = s1 < w ? s1 : w;
        if (pc1 <= pc0)
            continue;
        for (int j = 0; j < nz; ++j) {
            for (int u = 0; u < ksize; ++u) {
                const int r = pr - u + c0;
                if (r < 0 || r >= h)
                    continue;
                const double *xrow = vol + ((size_t)j * h + r) * w;
                /* voxel columns s whose taps reach [pc0, pc1) */
                const int sa = pc0 - c0 > 0 ? pc0 - c0 : 0;
                const int sb = pc1 - 1 + c0 < w - 1 ? pc1 - 1 + c0 : w - 1;
                for (int s = sa; s <= sb; ++s) {
                    const double xv = xrow[s];
                    if (xv == 0.0)
                        continue;
                    const float *k = psf + psf_index(nnum, ksize, j, r % nnum, s % nnum) +
                                     (size_t)u * ksize;
                    /* taps v with ps = s + v - c0 in [pc0, pc1) */
                    int va = pc0 - s + c0, vb = pc1 - s + c0;
                    if (va < 0)
                        va = 0;
                    if (vb > ksize)
                        vb = ksize;
                    double *o = orow + (s - c0 - s0);
                    for (int v = va; v < vb; ++v)
                        o[v] += xv * (double)k[v];
                }
            }
        }
    }
    return 0;
}

/* One back-projected voxel (j, r, s): correlate the image with the PSF of the
 * voxel's own depth and phase, centred on the voxel's pixel. */
static double backward_voxel(int nnum, int ksize, int h, int w,
                             const float *psf, const double *img, int j, int r, int s)
{
    const int c0 = (ksize - 1) / 2;
    const float *k = psf + psf_index(nnum, ksize, j, r % nnum, s % nnum);
    double sum = 0.0;
    for (int u = 0; u < ksize; ++u) {
        const int pr = r + u - c0;
        if (pr < 0 || pr >= h)
            continue;
        for (int v = 0; v < ksize; ++v) {
            const int ps = s + v - c0;
            if (ps < 0 || ps >= w)
                continue;
            sum += img[(size_t)pr * w + ps] * (double)k[(size_t)u * ksize + v];
        }
    }
    return sum;
}

/* Back projection (adjoint of oracle_forward) of the whole image. */
int oracle_backward(int nnum, int nz, int ksize, int h, int w,
                    const float *psf, const double *img, double *vol)
{
    if (nnum < 1 || nz < 1 || ksize < 1 || (ksize & 1) == 0 || h < 0 || w < 0)
        return -1;
    long rows = (long)nz * h;
#pragma omp parallel for schedule(static)
    for (long jr = 0; jr < rows; ++jr) {
        const int j = (int)(jr / h), r = (int)(jr % h);
        for (int s = 0; s < w; ++s)
            vol[((size_t)j * h + r) * w + s] = backward_voxel(nnum, ksize, h, w, psf, img, j, r, s);
    }
    return 0;
}

/* Back projection evaluated only at the listed voxels (j[i], r[i], s[i]). */
int oracle_backward_at(int nnum, int nz, int ksize, int h, int w,
                       const float *psf, const double *img,
                       long npts, const int *jj, const int *rr, const int *ss, double *out)
{
    if (nnum < 1 || nz < 1 || ksize < 1 || (ksize & 1) == 0)
        return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (long i = 0; i < npts; ++i)
        out[i] = backward_voxel(nnum, ksize, h, w, psf, img, jj[i], rr[i], ss[i]);
    return 0;
}

/* Number of threads the routines above use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
