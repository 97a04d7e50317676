// Stage 2: heterodyne beat signal and spectrogram (gfx950).
//
// The detector current is the square of the reference field plus the
// scattered fields (eq. 2); only the reference-scattered cross term survives
// the detector bandwidth (eq. 3).  With the reference amplitude 1/2, a
// detected packet of weight w, apparent velocity v and random phase phi0
// contributes sqrt(w) cos(2 pi (f t + phi0)) with beat frequency
// f = 2 v / lambda.  Frame k of the time-resolved cloud owns the samples
// [floor(k N/F), floor((k+1) N/F)) of the record.  The spectrogram is the
// magnitude of a windowed discrete Fourier transform swept over the record
// (Sec. I, Fig. 1): periodic Hann window of nfft samples every hop samples.
//
// Kernels:
//   synth_partial   one block per (frame, chunk of list entries): entries are
//                   staged in LDS and every thread accumulates a run of
//                   consecutive samples; at the run's first sample the phase
//                   f n / fs + phi0 is formed with an FP64 fused multiply-add
//                   and reduced to [0,1) in FP64 (records reach tens of
//                   thousands of cycles), its cosine and sine taken in FP32
//                   on the revolution-argument hardware unit; each further
//                   sample of the run rotates that pair by the entry's phase
//                   step per sample (cos and sin of 2 pi frac(f / fs), formed
//                   in FP64 when the entry is staged);
//   synth_reduce    sums the per-chunk partials in fixed order (deterministic);
//   stft_kernel     one block per window: real FFT of nfft points through an
//                   nfft/2-point complex Stockham FFT in LDS (radix 4, one
//                   radix-2 stage when needed) and the split step, then |X|.
#include "pdv_device.h"
#include "pdv_internal.h"

namespace pdv {

struct SynthFrame {
    uint64_t entry_begin;    // first entry of the frame in the entry array
    uint32_t n_entries;      // entries kept for the frame
    int32_t s_begin;         // first sample owned by the frame
    int32_t s_count;         // samples owned by the frame
    int32_t pad;
};

constexpr int SYNTH_CHUNK = 1024;       // entries staged per block
constexpr int SYNTH_THREADS = 128;
constexpr int SYNTH_RUN = 4;            // consecutive samples per thread and pass

// NQ consecutive samples per thread, starting at base + NQ x thread, over
// the staged entries; a thread whose run starts past the frame's samples
// has nothing to do.
template <int NQ>
__device__ __forceinline__ void synth_samples(const SynthFrame& F, int base, int ne, const double* s_r,
                                              const double* s_ph, const float* s_a, const float2* s_rot,
                                              float* out) {
    const int j0 = base + (int)threadIdx.x * NQ;
    if (j0 >= F.s_count) return;
    const double n0 = (double)(F.s_begin + j0);
    float acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.f;
    for (int i = 0; i < ne; ++i) {
        // fractional cycles in one v_fract_f64 (x - floor(x), exact; its
        // clamp below 1 only matters where the FP32 rounding gives 1 anyway)
        const float cyc = (float)__builtin_amdgcn_fract(fma(s_r[i], n0, s_ph[i]));
        const float a = s_a[i];
        float c = __builtin_amdgcn_cosf(cyc);
        acc[0] = fmaf(a, c, acc[0]);
        if constexpr (NQ > 1) {
            float sn = __builtin_amdgcn_sinf(cyc);
            const float2 rot = s_rot[i];
#pragma unroll
            for (int q = 1; q < NQ; ++q) {
                const float c2 = fmaf(c, rot.x, -sn * rot.y);
                sn = fmaf(c, rot.y, sn * rot.x);
                c = c2;
                acc[q] = fmaf(a, c, acc[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (j0 + q < F.s_count) out[j0 + q] = acc[q];
    }
}

// Accumulate sqrt(w) cos(2 pi frac(r n + phi)) for the frame's samples over
// one chunk of entries; r = 2 v / (lambda fs) cycles per sample.  A thread
// takes a run of up to SYNTH_RUN consecutive samples per pass (sharing each
// entry read and one exact phase); the run length is cut to what the frame's
// remaining samples need.
__global__ void __launch_bounds__(SYNTH_THREADS)
synth_partial_kernel(const SynthFrame* __restrict__ frames, const ListEntry* __restrict__ entries,
                     double two_over_lambda_fs, int n_chunks, int max_samples, float* __restrict__ partial) {
    __shared__ double s_r[SYNTH_CHUNK];
    __shared__ double s_ph[SYNTH_CHUNK];
    __shared__ float s_a[SYNTH_CHUNK];
    __shared__ float2 s_rot[SYNTH_CHUNK];
    const int f = blockIdx.x;
    const int ch = blockIdx.y;
    const SynthFrame F = frames[f];
    const int e0 = ch * SYNTH_CHUNK;
    int ne = (int)F.n_entries - e0;
    ne = ne < 0 ? 0 : (ne > SYNTH_CHUNK ? SYNTH_CHUNK : ne);
    for (int i = threadIdx.x; i < ne; i += blockDim.x) {
        const ListEntry E = entries[F.entry_begin + (uint64_t)(e0 + i)];
        const double r = E.v * two_over_lambda_fs;
        s_r[i] = r;
        double sn, cs;
        sincospi(2.0 * (r - floor(r)), &sn, &cs);
        s_rot[i] = make_float2((float)cs, (float)sn);
        s_ph[i] = (double)E.phase * 2.3283064365386963e-10;   // 2^-32
        s_a[i] = sqrtf(E.w);
    }
    __syncthreads();
    float* out = partial + ((uint64_t)f * n_chunks + ch) * (uint64_t)max_samples;
    for (int base = 0; base < F.s_count; base += SYNTH_RUN * SYNTH_THREADS) {
        const int left = F.s_count - base;
        const int nq = left >= SYNTH_RUN * SYNTH_THREADS ? SYNTH_RUN : (left + SYNTH_THREADS - 1) / SYNTH_THREADS;
        if (nq == 4) synth_samples<4>(F, base, ne, s_r, s_ph, s_a, s_rot, out);
        else if (nq == 3) synth_samples<3>(F, base, ne, s_r, s_ph, s_a, s_rot, out);
        else if (nq == 2) synth_samples<2>(F, base, ne, s_r, s_ph, s_a, s_rot, out);
        else synth_samples<1>(F, base, ne, s_r, s_ph, s_a, s_rot, out);
    }
}

__global__ void synth_reduce_kernel(const SynthFrame* __restrict__ frames, int n_chunks, int max_samples,
                                    const float* __restrict__ partial, float* __restrict__ signal) {
    const int f = blockIdx.x;
    const SynthFrame F = frames[f];
    const int used = F.n_entries == 0 ? 0 : (int)((F.n_entries + SYNTH_CHUNK - 1) / SYNTH_CHUNK);
    for (int j = threadIdx.x; j < F.s_count; j += blockDim.x) {
        float s = 0.f;
        for (int c = 0; c < used; ++c) s += partial[((uint64_t)f * n_chunks + c) * (uint64_t)max_samples + j];
        signal[F.s_begin + j] = s;
    }
}

// ---------------------------------------------------------------------------
// STFT
// ---------------------------------------------------------------------------
struct F2 {
    float x, y;
};
__device__ __forceinline__ F2 f2(float a, float b) { return F2{a, b}; }
__device__ __forceinline__ F2 cadd(F2 a, F2 b) { return f2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ F2 csub(F2 a, F2 b) { return f2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ F2 cmul(F2 a, F2 b) { return f2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ F2 cmul_mi(F2 a) { return f2(a.y, -a.x); }   // a * (-i)

// Twiddle and window tables (FP64-computed, stored FP32):
//   tw[m]   = exp(-2 pi i m / n) for the n-point complex FFT, m < n;
//   tr[k]   = exp(-2 pi i k / N) for the real split step, k <= n (N = 2n);
//   win[i]  = 0.5 - 0.5 cos(2 pi i / N), periodic Hann.
__global__ void stft_tables_kernel(int nfft, F2* tw, F2* tr, float* win) {
    const int n = nfft / 2;
    const double PI2 = 6.283185307179586476925286766559;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nfft; i += gridDim.x * blockDim.x) {
        win[i] = (float)(0.5 - 0.5 * cos(PI2 * (double)i / (double)nfft));
        if (i < n) {
            double sn, cs;
            sincos(-PI2 * (double)i / (double)n, &sn, &cs);
            tw[i] = f2((float)cs, (float)sn);
        }
        if (i <= n) {
            double sn, cs;
            sincos(-PI2 * (double)i / (double)nfft, &sn, &cs);
            tr[i] = f2((float)cs, (float)sn);
        }
    }
}

// One block per window; LDS holds two n-point complex buffers (ping-pong).
__global__ void __launch_bounds__(1024)
stft_kernel(const float* __restrict__ signal, int nfft, int hop, const F2* __restrict__ tw,
            const F2* __restrict__ tr, const float* __restrict__ win, float* __restrict__ map) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int n = nfft / 2;
    F2* A = (F2*)smem;
    F2* B = A + n;
    const int m = blockIdx.x;
    const float* x = signal + (uint64_t)m * hop;
    const int tid = threadIdx.x, nt = blockDim.x;
    // pack even/odd windowed samples as complex values
    for (int j = tid; j < n; j += nt) A[j] = f2(win[2 * j] * x[2 * j], win[2 * j + 1] * x[2 * j + 1]);
    __syncthreads();
    F2* src = A;
    F2* dst = B;
    int Ns = 1;
    // radix-4 Stockham stages
    while (Ns * 4 <= n) {
        const int q = n / 4;
        const int step = n / (Ns * 4);       // twiddle stride for this stage
        for (int j = tid; j < q; j += nt) {
            const int kk = j % Ns;
            F2 v0 = src[j], v1 = src[j + q], v2 = src[j + 2 * q], v3 = src[j + 3 * q];
            if (kk) {
                v1 = cmul(v1, tw[(kk * step) % n]);
                v2 = cmul(v2, tw[(2 * kk * step) % n]);
                v3 = cmul(v3, tw[(3 * kk * step) % n]);
            }
            // 4-point DFT (forward, exp(-2 pi i ...))
            const F2 s02 = cadd(v0, v2), d02 = csub(v0, v2);
            const F2 s13 = cadd(v1, v3), d13 = cmul_mi(csub(v1, v3));
            const int o = (j / Ns) * Ns * 4 + kk;
            dst[o] = cadd(s02, s13);
            dst[o + Ns] = cadd(d02, d13);
            dst[o + 2 * Ns] = csub(s02, s13);
            dst[o + 3 * Ns] = csub(d02, d13);
        }
        __syncthreads();
        F2* t = src; src = dst; dst = t;
        Ns *= 4;
    }
    // one radix-2 stage when n is 2 x a power of 4
    if (Ns < n) {
        const int h = n / 2;
        const int step = n / (Ns * 2);
        for (int j = tid; j < h; j += nt) {
            const int kk = j % Ns;
            F2 v0 = src[j], v1 = src[j + h];
            if (kk) v1 = cmul(v1, tw[(kk * step) % n]);
            const int o = (j / Ns) * Ns * 2 + kk;
            dst[o] = cadd(v0, v1);
            dst[o + Ns] = csub(v0, v1);
        }
        __syncthreads();
        F2* t = src; src = dst; dst = t;
        Ns *= 2;
    }
    // split step: X[k] = (Z[k] + conj(Z[n-k]))/2 - i W^k (Z[k] - conj(Z[n-k]))/2
    float* out = map + (uint64_t)m * (uint64_t)(n + 1);
    for (int k = tid; k <= n; k += nt) {
        const F2 zk = src[k == n ? 0 : k];
        const F2 zc = src[(n - k) % n];
        const F2 zcc = f2(zc.x, -zc.y);
        const F2 e = f2(0.5f * (zk.x + zcc.x), 0.5f * (zk.y + zcc.y));
        const F2 d = f2(0.5f * (zk.x - zcc.x), 0.5f * (zk.y - zcc.y));
        const F2 od = cmul(tr[k], cmul_mi(d));
        const F2 X = cadd(e, od);
        out[k] = sqrtf(X.x * X.x + X.y * X.y);
    }
}

// ---- host launchers ----
hipError_t launch_synth(hipStream_t s, int n_frames, const void* frames, const ListEntry* entries, double r_scale,
                        int n_chunks, int max_samples, float* partial, float* signal) {
    if (n_frames <= 0) return hipSuccess;
    if (n_chunks > 0) {
        hipLaunchKernelGGL(synth_partial_kernel, dim3(n_frames, n_chunks), dim3(SYNTH_THREADS), 0, s,
                           (const SynthFrame*)frames, entries, r_scale, n_chunks, max_samples, partial);
    }
    hipLaunchKernelGGL(synth_reduce_kernel, dim3(n_frames), dim3(256), 0, s, (const SynthFrame*)frames, n_chunks,
                       max_samples, partial, signal);
    return hipGetLastError();
}

hipError_t launch_stft(hipStream_t s, const float* signal, int n_windows, int nfft, int hop, void* tw, void* tr,
                       float* win, float* map, bool build_tables) {
    if (build_tables) {
        hipLaunchKernelGGL(stft_tables_kernel, dim3((nfft + 255) / 256), dim3(256), 0, s, nfft, (F2*)tw, (F2*)tr,
                           win);
    }
    if (n_windows > 0) {
        const int lds = nfft * (int)sizeof(F2);   // two buffers of nfft/2 complex values
        hipLaunchKernelGGL(stft_kernel, dim3(n_windows), dim3(nfft >= 2048 ? 1024 : nfft / 2), lds, s, signal,
                           nfft, hop, (const F2*)tw, (const F2*)tr, win, map);
    }
    return hipGetLastError();
}

int synth_chunk() { return SYNTH_CHUNK; }
size_t synth_frame_bytes() { return sizeof(SynthFrame); }

}  // namespace pdv
