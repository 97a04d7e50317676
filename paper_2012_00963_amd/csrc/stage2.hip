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
//   synth_tile      one wave per (sample tile, frame, group of entry chunks):
//                   the group's entries are staged in LDS a chunk at a time
//                   and every lane accumulates a run of consecutive samples
//                   of the tile; at the run's first sample the phase
//                   f n / fs + phi0 is formed with an FP64 fused multiply-add
//                   and reduced to [0,1) in FP64 (records reach tens of
//                   thousands of cycles), its cosine and sine taken in FP32
//                   on the revolution-argument hardware unit; the further
//                   samples of the run follow from the three-term recurrence
//                   of cos(x + q theta) in Reinsch's difference form
//                   (d += -4 sin^2(theta/2) c, c += d: two operations per
//                   sample, accurate for small steps theta), whose constants
//                   are formed in FP64 when the entry is staged.  With one
//                   group the block writes the record itself; otherwise each
//                   group writes a partial record;
//   synth_reduce    sums the groups' partial records in group order
//                   (deterministic);
//   stft_kernel     one block per window: real FFT of nfft points through an
//                   nfft/2-point complex Stockham FFT in LDS (radix 4, one
//                   radix-2 stage when needed) and the split step, then |X|.
#include <algorithm>
#include <mutex>

#include "pdv_device.h"
#include "pdv_internal.h"

namespace pdv {

// Partial records of the allocation-free synthesis entry point: a static
// array in every device's copy of the code object, held until the process
// ends.  Host code never uses the array's name as an address: each device's
// address comes from hipGetSymbolAddress at context creation.
static __device__ __align__(256) float scratch[SYNTH_PARTIAL_MAX_FLOATS];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch[SCRATCH_MAX_DEVICES] = {};
}  // namespace

// With `device` current: look up this device's address of the static
// scratch (once per device).
hipError_t synth_scratch_init(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = (float*)p;
    return hipSuccess;
}

// The device's scratch address, or nullptr before synth_scratch_init.
float* synth_scratch(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[device];
}

constexpr int SYNTH_CHUNK = 256;        // entries staged in LDS at a time (8 KB)
constexpr int SYNTH_THREADS = 64;       // one wave per block
constexpr int SYNTH_GROUPS = 8;         // lane groups, each taking every eighth entry
constexpr int SYNTH_LANES = SYNTH_THREADS / SYNTH_GROUPS;
constexpr int SYNTH_RUN = 64;           // consecutive samples per lane, at most
constexpr int SYNTH_TILE = SYNTH_RUN * SYNTH_LANES;

// Where the entries come from: an array of ListEntry records (lists written
// by the transport, or packed from host arrays), or, with rec null, three
// separate arrays.
struct EntrySrc {
    const ListEntry* rec;
    const float* w;
    const double* v;
    const uint32_t* phase;
};

__device__ __forceinline__ void load_entry(const EntrySrc& src, uint64_t i, float& w, double& v, uint32_t& ph) {
    if (src.rec) {
        const ListEntry E = src.rec[i];
        w = E.w;
        v = E.v;
        ph = E.phase;
    } else {
        w = src.w[i];
        v = src.v[i];
        ph = src.phase[i];
    }
}

// The chunks [c0, c1) of frame entries starting at e_begin (n_entries in
// all), accumulated over the NQ consecutive samples j0 .. j0 + NQ - 1 of the
// frame (absolute sample index n0 for j0).  The eight groups of eight lanes
// cover the same samples and take every eighth entry (lanes l, l + 8, ...,
// l + 56 hold the eight parts of one run's sums), so a lane's run is eight
// times as long as one wave over the tile would give it, and the starting
// phase of a run, its costly part, is paid once per NQ samples.  Every lane
// takes part in the staging; lanes whose run starts past the frame's samples
// only stage.
//
// Staged per entry: rp = (r, phi0), r = f / fs in cycles per sample, and
// st = (a, s a, k, sin t) with a = sqrt(w).  The step per sample is
// theta = 2 pi frac(r); where cos(theta) < 0 the recurrence runs with
// t = theta - pi and s = -1 (cos(x + q theta) = (-1)^q cos(x + q t)), else
// with t = theta and s = 1, so that |t| <= pi/2 and k = 4 sin^2(t/2) keeps
// the step accurate.  The run's samples: c_0 = cos x from the hardware unit,
// d_0 = c_0 - cos(x - t) = c_0 k/2 - sin x sin t, then d_{q+1} = d_q - k c_q
// and c_{q+1} = c_q + d_{q+1}; sample q adds a c_q (q even) or s a c_q (q odd).
// A lane group takes two of its entries per pass (an absent second entry
// has zero amplitude), so that their two recurrences interleave.
template <int NQ>
__device__ __forceinline__ void synth_tile(const EntrySrc& src, uint64_t e_begin, uint64_t n_entries, int c0, int c1,
                                           double r_scale, double n0, bool active, float* acc, double2* s_rp,
                                           float4* s_st) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.f;
    const int grp = (int)(threadIdx.x / SYNTH_LANES);
    for (int ch = c0; ch < c1; ++ch) {
        const uint64_t e0 = (uint64_t)ch * SYNTH_CHUNK;
        const int ne = (int)(n_entries - e0 < (uint64_t)SYNTH_CHUNK ? n_entries - e0 : (uint64_t)SYNTH_CHUNK);
        __syncthreads();            // the previous chunk's entries are no longer read
        // one entry at a time: the run's sums stay live across the staging
#pragma unroll 1
        for (int i = threadIdx.x; i < ne; i += blockDim.x) {
            float w;
            double v;
            uint32_t ph;
            load_entry(src, e_begin + e0 + (uint64_t)i, w, v, ph);
            const double r = v * r_scale;
            // the step in half cycles, in (-1, 1]
            double h = 2.0 * (r - floor(r));
            h = h > 1.0 ? h - 2.0 : h;
            // shifted by one half cycle where |h| > 1/2 (cos(theta) < 0)
            const bool flip = h > 0.5 || h < -0.5;
            const double t = flip ? (h > 0.0 ? h - 1.0 : h + 1.0) : h;
            double sh, ch_;
            sincospi(0.5 * t, &sh, &ch_);
            const float a = sqrtf(w);
            s_rp[i] = make_double2(r, (double)ph * 2.3283064365386963e-10);   // 2^-32
            // sin t = 2 sin(t/2) cos(t/2); k = 4 sin^2(t/2)
            s_st[i] = make_float4(a, flip ? -a : a, (float)(4.0 * sh * sh), (float)(2.0 * sh * ch_));
        }
        __syncthreads();
        if (!active) continue;
        for (int i = grp; i < ne; i += 2 * SYNTH_GROUPS) {
            const int i2 = i + SYNTH_GROUPS < ne ? i + SYNTH_GROUPS : i;
            const double2 rpA = s_rp[i], rpB = s_rp[i2];
            const float4 stA = s_st[i];
            float4 stB = s_st[i2];
            if (i2 == i) stB.x = stB.y = 0.f;
            // fractional cycles in one v_fract_f64 (x - floor(x), exact; its
            // clamp below 1 only matters where the FP32 rounding gives 1 anyway)
            const float cyA = (float)__builtin_amdgcn_fract(fma(rpA.x, n0, rpA.y));
            const float cyB = (float)__builtin_amdgcn_fract(fma(rpB.x, n0, rpB.y));
            float cA = __builtin_amdgcn_cosf(cyA), cB = __builtin_amdgcn_cosf(cyB);
            acc[0] = fmaf(stA.x, cA, acc[0]);
            acc[0] = fmaf(stB.x, cB, acc[0]);
            if constexpr (NQ > 1) {
                float dA = fmaf(0.5f * stA.z, cA, -__builtin_amdgcn_sinf(cyA) * stA.w);
                float dB = fmaf(0.5f * stB.z, cB, -__builtin_amdgcn_sinf(cyB) * stB.w);
#pragma unroll
                for (int q = 1; q < NQ; ++q) {
                    dA = fmaf(-stA.z, cA, dA);
                    dB = fmaf(-stB.z, cB, dB);
                    cA += dA;
                    cB += dB;
                    acc[q] = fmaf((q & 1) ? stA.y : stA.x, cA, acc[q]);
                    acc[q] = fmaf((q & 1) ? stB.y : stB.x, cB, acc[q]);
                }
            }
        }
    }
}

// One lane's run: the sums over the group's entries, the other lane groups'
// sums added onto the first group's (every lane takes part), and the first
// group's store of the run's samples below s_count.
template <int NQ>
__device__ __forceinline__ void synth_run(const EntrySrc& src, uint64_t e_begin, uint64_t n_entries, int c0, int c1,
                                          double r_scale, double n0, bool active, double2* s_rp, float4* s_st,
                                          float* out, int j0, int s_count) {
    float acc[NQ];
    synth_tile<NQ>(src, e_begin, n_entries, c0, c1, r_scale, n0, active, acc, s_rp, s_st);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int m = SYNTH_THREADS / 2; m >= SYNTH_LANES; m >>= 1) acc[q] += __shfl_xor(acc[q], m, 64);
    }
    if (!active || threadIdx.x >= SYNTH_LANES) return;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (j0 + q < s_count) out[j0 + q] = acc[q];
}

// The run of exactly nq samples (1 <= nq <= NQ): every run length has its
// own unrolled code, so no sample slot is computed and thrown away.
template <int NQ>
__device__ __forceinline__ void synth_dispatch(int nq, const EntrySrc& src, uint64_t e_begin, uint64_t n_entries,
                                               int c0, int c1, double r_scale, double n0, bool active,
                                               double2* s_rp, float4* s_st, float* out, int j0, int s_count) {
    if constexpr (NQ > 1) {
        if (nq < NQ) {
            synth_dispatch<NQ - 1>(nq, src, e_begin, n_entries, c0, c1, r_scale, n0, active, s_rp, s_st, out, j0,
                                   s_count);
            return;
        }
    }
    synth_run<NQ>(src, e_begin, n_entries, c0, c1, r_scale, n0, active, s_rp, s_st, out, j0, s_count);
}

// Frame f owns samples [floor(f N / F), floor((f+1) N / F)) and the entries
// [fbeg[f], fend[f]).  Block (tile, frame, group) accumulates the tile's
// SYNTH_TILE samples over the group's entry chunks: group g takes chunks
// [g cpg, (g+1) cpg), the last group every chunk from (G-1) cpg on.  Lane l
// and lanes l + 8, ..., l + 56 take the run of nq <= SYNTH_RUN consecutive
// samples from tile sample (l mod 8) x nq, nq cut to what the tile's
// remaining samples need.  With one group the block writes the record;
// otherwise partial[(f G + g) max_samples + j] for the frame's sample j.
__global__ void __launch_bounds__(SYNTH_THREADS)
synth_tile_kernel(const uint64_t* __restrict__ fbeg, const uint64_t* __restrict__ fend, EntrySrc src,
                  double r_scale, int n_frames, int n_samples, int n_groups, int cpg, int max_samples,
                  float* __restrict__ partial, float* __restrict__ signal) {
    __shared__ double2 s_rp[SYNTH_CHUNK];
    __shared__ float4 s_st[SYNTH_CHUNK];
    const int f = blockIdx.y;
    const int g = blockIdx.z;
    const int64_t s_begin = (int64_t)f * n_samples / n_frames;
    const int s_count = (int)((int64_t)(f + 1) * n_samples / n_frames - s_begin);
    const int tile_base = blockIdx.x * SYNTH_TILE;
    if (tile_base >= s_count) return;                      // uniform over the block
    const uint64_t e_begin = fbeg[f];
    const uint64_t e_end = fend[f];
    const uint64_t n_entries = e_end > e_begin ? e_end - e_begin : 0;
    const int used = (int)((n_entries + SYNTH_CHUNK - 1) / SYNTH_CHUNK);
    int c0 = g * cpg;
    int c1 = g == n_groups - 1 ? used : c0 + cpg;
    c0 = c0 < used ? c0 : used;
    c1 = c1 < used ? c1 : used;
    const int left = s_count - tile_base;
    const int nq = left >= SYNTH_TILE ? SYNTH_RUN : (left + SYNTH_LANES - 1) / SYNTH_LANES;
    const int j0 = tile_base + (int)(threadIdx.x & (SYNTH_LANES - 1)) * nq;
    const bool active = j0 < s_count;
    const double n0 = (double)(s_begin + j0);
    float* out = n_groups == 1 ? signal + s_begin : partial + ((uint64_t)f * n_groups + g) * (uint64_t)max_samples;
    synth_dispatch<SYNTH_RUN>(nq, src, e_begin, n_entries, c0, c1, r_scale, n0, active, s_rp, s_st, out, j0,
                              s_count);
}

__global__ void synth_reduce_kernel(int n_frames, int n_samples, int n_groups, int max_samples,
                                    const float* __restrict__ partial, float* __restrict__ signal) {
    const int f = blockIdx.y;
    const int64_t s_begin = (int64_t)f * n_samples / n_frames;
    const int s_count = (int)((int64_t)(f + 1) * n_samples / n_frames - s_begin);
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= s_count) return;
    const float* p = partial + (uint64_t)f * n_groups * (uint64_t)max_samples + j;
    float s = 0.f;
    for (int g = 0; g < n_groups; ++g) s += p[(uint64_t)g * max_samples];
    signal[s_begin + j] = s;
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

// Work split of a beat synthesis; the same for every entry point, so the
// summation order (and the FP32 record) depends only on the frames, their
// largest entry count and the record length.
SynthPlan synth_plan(int n_frames, int n_samples, uint64_t max_entries) {
    SynthPlan P;
    P.max_samples = n_frames > 0 ? (int)(((int64_t)n_samples + n_frames - 1) / n_frames) : 0;
    if (P.max_samples < 1) P.max_samples = 1;
    P.tiles = (P.max_samples + SYNTH_TILE - 1) / SYNTH_TILE;
    const uint64_t used = (max_entries + SYNTH_CHUNK - 1) / SYNTH_CHUNK;
    P.n_groups = 1;
    P.cpg = used > 0 ? (int)std::min<uint64_t>(used, 0x7fffffff) : 1;
    if (used > 1 && n_frames > 0) {
        const uint64_t base = (uint64_t)n_frames * (uint64_t)P.tiles;
        uint64_t G = (SYNTH_TARGET_BLOCKS + base - 1) / base;
        G = std::min<uint64_t>(G, used);
        const uint64_t cap = SYNTH_PARTIAL_MAX_FLOATS / ((uint64_t)n_frames * (uint64_t)P.max_samples);
        G = std::min<uint64_t>(G, cap);
        if (G >= 2) {
            const uint64_t cpg = (used + G - 1) / G;
            P.cpg = (int)cpg;
            P.n_groups = (int)((used + cpg - 1) / cpg);
        }
    }
    P.partial_floats = P.n_groups > 1 ? (uint64_t)n_frames * (uint64_t)P.n_groups * (uint64_t)P.max_samples : 0;
    return P;
}

// Entry ranges of frames whose lists sit at fixed capacity: frame f's list
// starts at f x capacity and holds min(count, capacity) entries.
__global__ void frame_ranges_kernel(int n_frames, uint64_t capacity, const uint64_t* __restrict__ counts,
                                    uint64_t* __restrict__ fbeg, uint64_t* __restrict__ fend) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_frames) return;
    const uint64_t c = counts[f];
    fbeg[f] = (uint64_t)f * capacity;
    fend[f] = (uint64_t)f * capacity + (c < capacity ? c : capacity);
}

void launch_frame_ranges(hipStream_t s, int n_frames, uint64_t capacity, const uint64_t* counts, uint64_t* fbeg,
                         uint64_t* fend) {
    if (n_frames <= 0) return;
    hipLaunchKernelGGL(frame_ranges_kernel, dim3((n_frames + 255) / 256), dim3(256), 0, s, n_frames, capacity, counts,
                       fbeg, fend);
}

hipError_t launch_synth(hipStream_t s, const SynthPlan& P, int n_frames, int n_samples, const uint64_t* fbeg,
                        const uint64_t* fend, const ListEntry* rec, const float* w, const double* v,
                        const uint32_t* phase, double r_scale, float* partial, float* signal) {
    if (n_frames <= 0 || n_samples <= 0) return hipSuccess;
    const EntrySrc src{rec, w, v, phase};
    const dim3 grid((unsigned)P.tiles, (unsigned)n_frames, (unsigned)P.n_groups);
    hipLaunchKernelGGL(synth_tile_kernel, grid, dim3(SYNTH_THREADS), 0, s, fbeg, fend, src, r_scale, n_frames,
                       n_samples, P.n_groups, P.cpg, P.max_samples, partial, signal);
    if (P.n_groups > 1)
        hipLaunchKernelGGL(synth_reduce_kernel, dim3((unsigned)((P.max_samples + 255) / 256), (unsigned)n_frames),
                           dim3(256), 0, s, n_frames, n_samples, P.n_groups, P.max_samples, partial, signal);
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


}  // namespace pdv
