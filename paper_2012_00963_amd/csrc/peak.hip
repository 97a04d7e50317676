// Peak analysis of velocity spectra (Sec. III.C): Fourier low-pass
// smoothing, peak position and relative curvature, and the ejecta's
// velocity-profile coefficient and optical thickness from the inverted peak
// relations (eq. 31 and eq. 34-35).
//
// One block per spectrum.  The n bin values, a table of the n-th roots of
// unity and the kept coefficients sit in LDS; the DFT coefficients A_k, B_k of the modes k <= K are
// plain sums over the bins (threads over k), the smoothed spectrum at the
// bin centres is the band-limited series (threads over bins), the largest
// value inside the search window is found by a block reduction, and Newton
// steps on the series' exact first and second derivatives locate the peak
// to within rounding.  All arithmetic is FP64.
#include <math.h>

#include "pdv_internal.h"

namespace pdv {

constexpr double PK_PI = 3.14159265358979323846;
constexpr int PK_THREADS = 256;
constexpr int PK_NEWTON = 12;

__device__ double pk_block_sum(double v, double* red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int off = PK_THREADS / 2; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// value (deriv 0), first or second derivative of the band-limited series at
// the continuous bin coordinate t; the block sums over the modes
__device__ double pk_series(const double* A, const double* B, int n, int keep, double t, int deriv, double* red) {
    double s = 0.0;
    for (int k = 1 + (int)threadIdx.x; k <= keep; k += PK_THREADS) {
        const double w = 2.0 * PK_PI * (double)k / (double)n;
        const double c = cos(w * t), si = sin(w * t);
        double term;
        if (deriv == 0) term = A[k] * c + B[k] * si;
        else if (deriv == 1) term = w * (-A[k] * si + B[k] * c);
        else term = -w * w * (A[k] * c + B[k] * si);
        s += 2.0 * term / (double)n;
    }
    s = pk_block_sum(s, red);
    if (deriv == 0) s += A[0] / (double)n;
    return s;
}

__global__ void __launch_bounds__(PK_THREADS)
peak_kernel(const double* __restrict__ spectra, int n, int keep, PeakJob J, double* __restrict__ smoothed,
            PeakOut* __restrict__ out) {
    extern __shared__ __align__(16) double pk_lds[];
    double* W = pk_lds;                 // n bin values
    double* tc = W + n;                 // cos(2 pi m / n)
    double* ts = tc + n;                // sin(2 pi m / n)
    double* A = ts + n;                 // A_k, k = 0..keep
    double* B = A + keep + 1;           // B_k
    __shared__ double red[PK_THREADS];
    __shared__ int ired[PK_THREADS];
    const int tid = threadIdx.x;
    const double* src = spectra + (uint64_t)blockIdx.x * n;
    for (int m = tid; m < n; m += PK_THREADS) {
        W[m] = src[m];
        const double ang = 2.0 * PK_PI * (double)m / (double)n;
        tc[m] = cos(ang);
        ts[m] = sin(ang);
    }
    __syncthreads();
    // DFT coefficients of the kept modes
    for (int k = tid; k <= keep; k += PK_THREADS) {
        double a = 0.0, b = 0.0;
        int m = 0;                      // (k b) mod n, advanced by k each bin
        for (int i = 0; i < n; ++i) {
            a += W[i] * tc[m];
            b += W[i] * ts[m];
            m += k;
            if (m >= n) m -= n;
        }
        A[k] = a;
        B[k] = b;
    }
    __syncthreads();
    // smoothed spectrum at the bin centres; best bin inside the window
    double best = -INFINITY;
    int best_i = n;
    for (int i = tid; i < n; i += PK_THREADS) {
        double s = 0.0;
        int m = 0;
        for (int k = 1; k <= keep; ++k) {
            m += i;
            m %= n;
            s += 2.0 * (A[k] * tc[m] + B[k] * ts[m]) / (double)n;
        }
        s += A[0] / (double)n;
        if (smoothed) smoothed[(uint64_t)blockIdx.x * n + i] = s;
        const double vc = J.v_lo + ((double)i + 0.5) * J.dv;
        if (vc >= J.search_lo && vc < J.search_hi && (s > best || (s == best && i < best_i))) {
            best = s;
            best_i = i;
        }
    }
    red[tid] = best;
    ired[tid] = best_i;
    __syncthreads();
    for (int off = PK_THREADS / 2; off > 0; off >>= 1) {
        if (tid < off) {
            const double o = red[tid + off];
            const int oi = ired[tid + off];
            if (o > red[tid] || (o == red[tid] && oi < ired[tid])) {
                red[tid] = o;
                ired[tid] = oi;
            }
        }
        __syncthreads();
    }
    const int b0 = ired[0];
    __syncthreads();
    PeakOut r;
    r.bin = b0;
    r.status = 0;
    // Newton steps on the series' derivative, kept inside [b0 - 1, b0 + 1]
    // and the window's bins; a best bin where the series is not concave is
    // no peak (status 1, position left at the bin)
    const double lo = fmax((double)b0 - 1.0, (double)J.wb0), hi = fmin((double)b0 + 1.0, (double)J.wb1);
    double t = (double)b0;
    const bool concave = pk_series(A, B, n, keep, t, 2, red) < 0.0;
    for (int it = 0; concave && it < PK_NEWTON; ++it) {
        const double d1 = pk_series(A, B, n, keep, t, 1, red);
        const double d2 = pk_series(A, B, n, keep, t, 2, red);
        if (!(d2 < 0.0)) break;
        double step = -d1 / d2;
        step = fmin(fmax(step, -0.5), 0.5);
        const double tn = fmin(fmax(t + step, lo), hi);
        if (tn == t) break;
        t = tn;
    }
    const double val = pk_series(A, B, n, keep, t, 0, red);
    const double d2 = pk_series(A, B, n, keep, t, 2, red);
    if (tid == 0) {
        r.t_peak = t;
        r.v_peak = J.v_lo + (t + 0.5) * J.dv;
        r.x_peak = r.v_peak / J.v_fs;
        r.value = val;
        r.rel_curvature = d2 / val * (J.v_fs / J.dv) * (J.v_fs / J.dv);
        if (concave && r.rel_curvature < 0.0) {
            r.beta = sqrt(-r.rel_curvature);
            r.tau0 = exp(r.beta * (r.x_peak - 1.0));
        } else {
            r.status = 1;
            r.beta = NAN;
            r.tau0 = NAN;
        }
        out[blockIdx.x] = r;
    }
}

// dynamic LDS of one block: bins, root table, coefficients
int peak_lds_bytes(int n, int keep) { return 8 * (3 * n + 2 * (keep + 1)); }

hipError_t launch_peak(hipStream_t s, int n_spectra, const double* spectra, int n, int keep, const PeakJob& J,
                       double* smoothed, PeakOut* out) {
    const int lds = peak_lds_bytes(n, keep);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&peak_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(peak_kernel, dim3(n_spectra), dim3(PK_THREADS), lds, s, spectra, n, keep, J, smoothed, out);
    return hipGetLastError();
}

}  // namespace pdv
