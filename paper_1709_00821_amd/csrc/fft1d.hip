// Recorded probe series and their FFT (the post-processing of the paper's
// section IV-B, which records the probe field over the run and Fourier
// transforms it), for gfx950.
//
// The series of row r holds E^m at its probe for m = 1 .. steps (entry m-1).
// The transform is the zero-padded DFT on nfft points (a power of 2 above
// steps), in the convention of the running DFT:
//   X_r[k] = dt sum_{m=1}^{steps} E^m exp(-j 2 pi k m / nfft),
// i.e. the running DFT's value at f_k = k / (nfft dt).
//
// Radix-2 Stockham autosort passes over global memory (ping-pong buffers, one
// launch a pass, natural order in and out; log2(nfft) passes), one thread a
// butterfly.  Pass with sub-transform length Ns (1, 2, 4, .., nfft/2): the
// butterfly j (0 <= j < nfft/2) reads a = x[j], b = x[j + nfft/2], turns b by
// exp(-j 2 pi (j mod Ns) / (2 Ns)) and writes a + b and a - b to positions
// (j / Ns) 2 Ns + (j mod Ns) and that + Ns.  The twiddle angle is formed as
// an exact fraction of pi (sincospi), so no twiddle rounds its argument.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace fdtdp {

// series[row][m0 + i] = samp[row][i] for i < count and m0 + i < R.
__global__ void k_series_copy(const double *samp, int SB, int64_t rows, int count, double *series, int64_t R,
                              int64_t m0)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * (int64_t)count) return;
    const int64_t row = t / count, i = t % count;
    if (m0 + i < R) series[row * R + m0 + i] = samp[row * SB + i];
}

void launch_series_copy(const double *samp, int SB, int64_t rows, int count, double *series, int64_t R,
                        int64_t m0, hipStream_t st)
{
    if (count <= 0 || rows <= 0 || m0 >= R) return;
    const int64_t tot = rows * (int64_t)count;
    hipLaunchKernelGGL(k_series_copy, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, samp, SB, rows,
                       count, series, R, m0);
}

// buf[row][m] = E^m (m = 1 .. steps), 0 at m = 0 and m > steps.
__global__ void k_fft_load(const double *series, int64_t R, int64_t rows, int64_t steps, int64_t nfft,
                           double2 *buf)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * nfft) return;
    const int64_t row = t / nfft, m = t % nfft;
    const double v = (m >= 1 && m <= steps) ? series[row * R + m - 1] : 0.0;
    buf[t] = make_double2(v, 0.0);
}

// One radix-2 Stockham pass of sub-transform length Ns over every row; the
// last pass (2 Ns = nfft) also scales by `scale` (dt).
__global__ void k_fft_pass(const double2 *src, double2 *dst, int64_t rows, int64_t nfft, int64_t Ns, double scale)
{
    const int64_t half = nfft >> 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * half) return;
    const int64_t row = t / half, j = t % half;
    const double2 *x = src + row * nfft;
    double2 *y = dst + row * nfft;
    const double2 a = x[j], b0 = x[j + half];
    const int64_t k = j % Ns;
    // exp(-j pi k / Ns)
    double s, c;
    sincospi(-(double)k / (double)Ns, &s, &c);
    const double2 b = make_double2(fmat(b0.x, c, -b0.y * s), fmat(b0.x, s, b0.y * c));
    const int64_t o = (j / Ns) * 2 * Ns + k;
    const double sc = (2 * Ns == nfft) ? scale : 1.0;
    y[o] = make_double2((a.x + b.x) * sc, (a.y + b.y) * sc);
    y[o + Ns] = make_double2((a.x - b.x) * sc, (a.y - b.y) * sc);
}

// The transform of every row into buf0 or buf1; returns the buffer holding it.
double2 *launch_fft(const double *series, int64_t R, int64_t rows, int64_t steps, int64_t nfft, double dt,
                    double2 *buf0, double2 *buf1, hipStream_t st)
{
    const int64_t tot = rows * nfft;
    hipLaunchKernelGGL(k_fft_load, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, series, R, rows,
                       steps, nfft, buf0);
    double2 *src = buf0, *dst = buf1;
    const int64_t bt = rows * (nfft >> 1);
    for (int64_t Ns = 1; Ns < nfft; Ns <<= 1) {
        hipLaunchKernelGGL(k_fft_pass, dim3((unsigned)((bt + 255) / 256)), dim3(256), 0, st, src, dst, rows,
                           nfft, Ns, dt);
        double2 *t = src;
        src = dst;
        dst = t;
    }
    return src;
}

}  // namespace fdtdp
