/*
 * pdv.h — C ABI of the MI355X PDV multiple-scattering Monte Carlo library
 * (libpdv.so, HIP for gfx950).
 *
 * The library simulates the photon Doppler velocimetry (PDV) spectrum of an
 * ejecta cloud in front of a moving free surface, following Shi et al.,
 * "Reconstruction and interpretation of photon Doppler velocimetry spectrum
 * for ejecta particles from shock-loaded sample in vacuum" (arXiv
 * 2012.00963):
 *   - the problem statement of Sec. II: particle cloud (velocity profile,
 *     eq. 20; size distribution, eq. 21; optical depth, eq. 7-8), particle
 *     optics (Mie, eq. 11-14, or a given phase function), probing wavelength,
 *     diffuse free surface, detector acceptance;
 *   - the Monte Carlo procedure of Sec. II.B (free flight, scatter/absorb,
 *     new direction, Doppler shift eq. 4 and 18, surface reflection, exit);
 *   - the output spectrum of eq. 19 (histogram of outgoing photons by
 *     apparent velocity) and the heterodyne spectrogram of eq. 1-3 and
 *     Sec. I (beat signal swept by a windowed discrete Fourier transform).
 *
 * Conventions for every entry point:
 *   - SI units: metres, seconds, m/s, radians.
 *   - The apparent velocity of a photon is v~ = c (omega - omega_r)/(2
 *     omega_r); a single straight back-scatter from a particle of speed V
 *     gives v~ = V.  Histograms are over v~.
 *   - All pointers in parameter and output structs are HOST pointers unless
 *     a field says "device".  Inputs are only read during the call; outputs
 *     are caller-owned and fully written before a blocking call returns.
 *   - Return value: PDV_OK (0) or a negative pdv_status.  No exception
 *     crosses the ABI.  pdv_last_error() gives a message for the last failed
 *     call on that context.  After PDV_EDEVICE the context is poisoned: every
 *     later call returns PDV_EDEVICE; destroy and recreate it.
 *   - One context per host thread, except the serving calls (pdv_submit,
 *     pdv_poll, pdv_cancel, pdv_serve_report), which are thread-safe.
 *   - Fixed-point tallies: weights are accumulated as unsigned 64-bit
 *     integers scaled by 2^32 (divide by 4294967296.0 for packet-weight
 *     units).  Integer sums are order independent, so results are bitwise
 *     reproducible whatever the launch shape, batching or partition.
 */
#ifndef PDV_H
#define PDV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PDV_ABI_VERSION 2

typedef enum {
    PDV_OK = 0,
    PDV_PENDING = 1,      /* pdv_poll: request not finished yet */
    PDV_EINVAL = -1,      /* invalid argument (message in pdv_last_error) */
    PDV_ENOMEM = -2,      /* device allocation failed or request exceeds the memory budget */
    PDV_EDEVICE = -3,     /* HIP error; the context is poisoned */
    PDV_EOVERFLOW = -4,   /* a detected list exceeded its capacity (results still valid, list truncated) */
    PDV_ECANCELLED = -5,  /* serving: request was cancelled */
    PDV_ESTATE = -6,      /* call not valid in the current state (e.g. serving not started) */
    PDV_ENOTFOUND = -7    /* serving: unknown ticket */
} pdv_status;

enum { PDV_DENSITY_UNIFORM = 0, PDV_DENSITY_EXP = 1, PDV_DENSITY_TABLE = 2 };
enum { PDV_PHASE_HG = 0, PDV_PHASE_TABLE = 1, PDV_PHASE_MIE = 2 };
enum { PDV_SURFACE_UNIFORM_THETA = 0, PDV_SURFACE_LAMBERT = 1 };
enum { PDV_WEIGHT_IMPLICIT = 0, PDV_WEIGHT_ANALOG = 1 };
enum { PDV_FP32 = 0, PDV_FP64 = 1 };

/* Flags of pdv_params.flags */
#define PDV_FLAG_CLASS_TALLIES 1u   /* also tally the single-scattering and surface-only classes */
/* w_fx, w2_fx (and class_fx) of this set's pdv_spectrum_out are device
 * pointers on the context's device (for example a torch tensor's data_ptr,
 * with the library loaded into the HIP runtime PyTorch uses, as the Python
 * binding does): the library writes the bins there on the context's stream
 * (the caller's, when one was given to pdv_create), device to device, and
 * has finished when the call returns; the scalar fields of pdv_spectrum_out
 * stay host memory.  Accepted by pdv_spectrum and pdv_spectrum_batch only
 * (pdv_spectrogram and pdv_submit reject it); a pointer that is not device
 * memory of the context's device gives PDV_EINVAL before any work. */
#define PDV_FLAG_DEVICE_OUTPUT 2u
/* Also score the next-event (peel-off) estimate of the detector tally into
 * pdv_spectrum_out.peel_fx: at every particle scattering and surface
 * reflection, the expected weight that leaves the top inside the detector
 * cone on the next flight (Beer-Lambert escape of eq. 7 times the share of
 * the scattering law, eq. 13-16, or of the surface law that points into the
 * cone, detector of eq. 19), scored at the apparent velocity after the event
 * (eq. 4), from one draw restricted to the directions that reach the cone
 * (its own Philox block, counter word 0 = event index | 2^31, so the
 * ordinary tally is unchanged).  Its expectation equals the detector tally;
 * for narrow cones its variance is far lower.  Accepted by pdv_spectrum and
 * pdv_spectrum_batch only. */
#define PDV_FLAG_PEEL 4u
/* Add this call's tallies and counters to what the (host) outputs already
 * hold instead of overwriting them: checkpoint and resume.  A run of packets
 * [0, N) split into calls over [0, k) and [k, N) (pid_begin = k,
 * n_packets = N - k, outputs carried over, for example saved to disk and
 * read back) equals one call over [0, N) bit for bit, because every packet
 * draws from its own random stream and the tallies are integer sums.  Not
 * with PDV_FLAG_DEVICE_OUTPUT (PDV_EINVAL).  Served requests accept it. */
#define PDV_FLAG_ACCUMULATE 8u

/*
 * One parameter set: the problem statement of Sec. II.
 *
 * Cloud (Sec. II.C): self-similar expansion z = v t, so the slab is described
 * in the velocity coordinate zeta in [v_bottom, v_top] and a particle at zeta
 * moves along the outward normal at speed zeta.  The slab is cut into
 * n_layers equal zeta-layers (Sec. II.B step 2 uses 1000) of constant
 * extinction; each layer's optical depth is tau_total times its share of
 * the column density:
 *   UNIFORM: constant density;
 *   EXP:     density proportional to exp(-(zeta - v_bottom)/v0) (eq. 20 with
 *            v0 = v_fs/beta);
 *   TABLE:   density[n_layers] (host), per-layer relative weights ordered
 *            from the bottom layer upwards.
 * tau_total is the normal extinction optical depth of the whole slab (eq. 7-8).
 *
 * Particle optics (eq. 11-14):
 *   HG:    Henyey-Greenstein phase function with asymmetry hg_g (|hg_g| < 1)
 *          and single-scattering albedo `albedo` (K_sca/K_ext);
 *   TABLE: phase[n_angles] (host), p(theta_j) at theta_j = j pi/(n_angles-1),
 *          any positive scale, with albedo `albedo`;
 *   MIE:   spheres of complex refractive index m_re + i m_im at `wavelength`,
 *          log-normal number distribution (eq. 21) with median d_median and
 *          width sigma_ln, truncated to [d_min, d_max], integrated over ln d
 *          with n_size_nodes Gauss-Legendre nodes; the albedo and the phase
 *          function (tabulated at n_angles angles) are size averages.
 *   The scattering angle is drawn from the integer CDF of the tabulated phase
 *   function (trapezoid cells of p sin(theta), uniform angle inside a cell).
 *
 * Free surface (Sec. II.B, after eq. 18): at zeta = v_bottom, moving at
 * v_surface, reflecting a fraction surface_albedo diffusely:
 *   UNIFORM_THETA: polar angle uniform over the upper hemisphere (the
 *                  paper's wording);  LAMBERT: cosine-law reflection.
 *
 * Detector: photons leaving the top within cone_half_angle of the normal
 * (pi/2 accepts every outgoing photon, as eq. 19 does) are histogrammed in
 * n_bins equal bins over [v_lo, v_hi); others go to the sinks.
 *
 * Transport: at most max_orders particle scatterings per packet (the next
 * interaction moves the remaining weight to the "truncated" sink).
 * weighting IMPLICIT multiplies the packet weight by the albedo at every
 * interaction; ANALOG absorbs the packet with probability 1 - albedo
 * (eq. 11 literally).  precision FP32 (FP32 transport, FP64 tallies) or FP64.
 *
 * Packets pid_begin .. pid_begin + n_packets - 1; packet pid, event k uses
 * the Philox4x32-10 block with counter (k, pid low, pid high, stream) and key
 * (seed low, seed high); the block with k = 0xFFFFFFFF gives the beat phase.
 */
typedef struct pdv_params {
    double wavelength;
    double v_bottom, v_top;
    int32_t density_kind;
    int32_t n_layers;
    double v0;
    const double* density;
    double tau_total;
    int32_t phase_kind;
    int32_t n_angles;
    double hg_g;
    double albedo;
    const double* phase;
    double m_re, m_im;
    double d_median, sigma_ln, d_min, d_max;
    int32_t n_size_nodes;
    int32_t surface_law;
    double v_surface, surface_albedo;
    double cone_half_angle;
    double v_lo, v_hi;
    int32_t n_bins;
    int32_t max_orders;
    int32_t weighting;
    int32_t precision;
    uint64_t n_packets;
    uint64_t pid_begin;
    uint64_t seed;
    uint32_t stream;
    uint32_t flags;
} pdv_params;

/* Sinks (weights x 2^32) in pdv_spectrum_out.sinks_fx */
enum { PDV_SINK_UNDER = 0, PDV_SINK_OVER = 1, PDV_SINK_UNDETECTED = 2,
       PDV_SINK_ABSORBED_PARTICLE = 3, PDV_SINK_ABSORBED_SURFACE = 4,
       PDV_SINK_TRUNCATED = 5, PDV_N_SINKS = 6 };

typedef struct pdv_counters {
    uint64_t packets;     /* packets transported */
    uint64_t collisions;  /* particle interactions (scattering or absorption) */
    uint64_t surface;     /* free-surface hits */
    uint64_t exits;       /* packets that left the top of the cloud */
    uint64_t detected;    /* exits inside the detector cone */
} pdv_counters;

/*
 * Output of one spectrum.  w_fx and w2_fx: caller-owned host arrays of
 * n_bins entries receiving sum(w) and sum(w^2) per bin (x 2^32); device
 * arrays instead when the set has PDV_FLAG_DEVICE_OUTPUT.  class_fx:
 * nullable; if given and PDV_FLAG_CLASS_TALLIES is set, 2*n_bins entries:
 * [0, n_bins) single-scattering paths (one particle scattering, no surface
 * hit), [n_bins, 2 n_bins) surface-only paths.  Conservation holds exactly:
 * sum(w_fx) + sum(sinks_fx) = n_packets * 2^32.  peel_fx: nullable; if
 * given and PDV_FLAG_PEEL is set, 2*n_bins entries (x 2^32, each score
 * rounded to the nearest 2^-32): [0, n_bins) the next-event estimate sum(c)
 * per bin, [n_bins, 2 n_bins) sum(c^2); peel_sinks_fx: its scores below and
 * above the bin range.
 */
typedef struct pdv_spectrum_out {
    uint64_t* w_fx;
    uint64_t* w2_fx;
    uint64_t* class_fx;
    uint64_t sinks_fx[PDV_N_SINKS];
    pdv_counters counters;
    double albedo;        /* single-scattering albedo used (Mie: size average) */
    double g;             /* mean cosine of the phase function used */
    uint64_t* peel_fx;
    uint64_t peel_sinks_fx[2];
} pdv_spectrum_out;

/* Launch options for batches; pass NULL for the tuned defaults. */
typedef struct pdv_launch_opts {
    int32_t block_size;          /* threads per block: 256, 512, 768 or 1024; 0 = default */
    int32_t blocks_per_cu;       /* persistent grid = blocks_per_cu x CUs; 0 = default */
    uint64_t packets_per_item;   /* work-item size; 0 = default (with one FP32 set of the tabulated kind and
                                    no lists, a persistent launch's waves take items by themselves, an
                                    eighth of a wave's share) */
    int32_t persistent;          /* 1 = persistent work queue, 0 = one block per item, -1 = default */
    int32_t use_graph;           /* 1 = capture and replay the batch as a hipGraph, 0 = direct launches */
    int32_t guide_bits;          /* search-guide cells 2^guide_bits staged in LDS, 11..14; 0 = the finest
                                    that keeps the launch's blocks resident (a table layout: results are
                                    bitwise the same for every value) */
    int32_t retire_batch;        /* finished lanes a wave collects before it tallies and refills them,
                                    1..64; 0 = default (FP32: 16, or 24 when detected lists are
                                    written; FP64: 1); results do not depend on it */
} pdv_launch_opts;

/*
 * Create a context on HIP device `device`.  mem_budget bounds the device
 * memory the context may hold (0 = 90% of free memory).  hip_stream: a
 * hipStream_t to run on (nullable: the context creates its own).
 * Errors: PDV_EINVAL (bad device or NULL out), PDV_EDEVICE (no device / HIP
 * failure; *out is still set so pdv_last_error can be read, then destroy it).
 */
int pdv_create(struct pdv_ctx** out, int device, uint64_t mem_budget, void* hip_stream);
void pdv_destroy(struct pdv_ctx* ctx);
/* Message of the last failed call on ctx (never NULL; "" if none). */
const char* pdv_last_error(const struct pdv_ctx* ctx);
/* ABI version and the HIP device count (without creating a context). */
int pdv_abi_version(void);
int pdv_device_count(int* count);

/*
 * Validate a parameter set without running it.  Returns PDV_OK or
 * PDV_EINVAL with the reason in pdv_last_error (ctx may be NULL: then the
 * reason is not kept).  Checks: 1 <= n_bins <= 4096, v_hi > v_lo, v_top >= v_bottom,
 * tau_total >= 0, 0 <= albedo, surface_albedo <= 1, |hg_g| < 1, cone in
 * (0, pi/2], 1 <= n_layers <= 4096, 16 <= n_angles <= 4096, Mie sizes
 * 0 < d_min < d_median, d_median < d_max, sigma_ln > 0, 8 <= n_size_nodes <= 1024,
 * 0 <= max_orders <= 100000, n_packets < 2^32 (fixed-point headroom: every
 * tally stays below 2^64).
 */
int pdv_validate(struct pdv_ctx* ctx, const pdv_params* p);

/*
 * Set tables alone (Sec. II.B eq. 7-8, 11-14; Sec. II.C eq. 20-21): builds
 * one parameter set's device tables -- the cumulative extinction depth of
 * each layer, and the phase CDF with its guide (tabulated law) or the
 * size-averaged Mie optics of the truncated log-normal -- and reports what
 * they hold, without transporting packets (n_packets is ignored).  The
 * tables are rebuilt by every spectrum call; this call is for inspecting
 * them (albedo and mean cosine of a Mie cloud, the realised optical depth).
 * info: caller-owned output.  Errors: PDV_EINVAL (invalid parameters, NULL
 * pointers), PDV_ESTATE (context without a device), PDV_EDEVICE.
 */
typedef struct {
    double albedo;        /* single-scattering albedo the transport uses (Mie: size-averaged K_sca/K_ext) */
    double g;             /* mean cosine of the sampled scattering law */
    double tau_total;     /* last cumulative layer depth of the FP64 table (equals p->tau_total up to rounding) */
    double tau_total_f32; /* the same depth in the FP32 table the FP32 transport reads */
    int32_t n_layers;
    int32_t n_cells;      /* angle cells of the phase CDF (n_angles - 1); 0 for Henyey-Greenstein */
} pdv_table_info;
int pdv_prepare(struct pdv_ctx* ctx, const pdv_params* p, pdv_table_info* info);

/*
 * One spectrum (blocking).  Builds the set's tables on the device (layer
 * depths; Mie size average and phase CDF, or HG constants), transports
 * n_packets packets and copies the tallies to `out`.
 */
int pdv_spectrum(struct pdv_ctx* ctx, const pdv_params* p, pdv_spectrum_out* out);

/*
 * n parameter sets in one persistent launch (blocking).  Sets may differ in
 * every field except precision (all FP32 or all FP64).  Work items of
 * packets_per_item packets are handed out largest set first; each block
 * stages one set's tables in LDS at a time.  outs[i] receives set i.
 * opts: nullable launch options.
 */
int pdv_spectrum_batch(struct pdv_ctx* ctx, const pdv_params* sets, int32_t n,
                       pdv_spectrum_out* outs, const pdv_launch_opts* opts);

/*
 * Spectrogram (Sec. I, eq. 1-3): n_frames frames of the cloud `p`
 * (self-similar expansion, so each frame is the same zeta-slab; frame k uses
 * stream p->stream + k and packets_per_frame packets).  Detected packets
 * (weight w, apparent velocity v~, phase phi0) of frame k feed the samples
 * [floor(k N/F), floor((k+1) N/F)) of a beat record of n_samples samples at
 * fs samples/s: s[n] = sum sqrt(w) cos(2 pi frac(f n / fs + phi0)),
 * f = 2 v~ / wavelength, phase in FP64.  The record is cut into windows of
 * nfft samples (periodic Hann) every hop samples; map receives
 * |DFT| of each window, n_windows x (nfft/2 + 1) floats, window-major.
 */
typedef struct pdv_sg_params {
    int32_t n_frames;
    int32_t nfft;                 /* power of two, 256 .. 8192 */
    int32_t hop;
    int32_t n_samples;
    uint64_t packets_per_frame;
    uint64_t list_capacity;       /* detected entries kept per frame */
    double fs;
} pdv_sg_params;

typedef struct pdv_sg_out {
    float* map;                   /* host, n_windows x (nfft/2+1); n_windows = (n_samples - nfft)/hop + 1 */
    float* signal;                /* nullable host [n_samples]: the beat record */
    uint64_t* frame_counts;       /* nullable host [n_frames]: detected entries per frame (before capping) */
    int32_t n_windows;            /* written */
    int32_t overflow;             /* written: 1 if some frame exceeded list_capacity */
    pdv_spectrum_out* spectrum;   /* nullable: tallies summed over all frames */
    /* nullable host arrays of n_frames x list_stride entries: the detected
     * list of frame k (weight, apparent velocity, phase word; phase in cycles
     * is phase / 2^32) fills [k list_stride, k list_stride + min(count_k,
     * list_stride, list_capacity)); order inside a frame is unspecified */
    float* list_w;
    double* list_v;
    uint32_t* list_phase;
    uint64_t list_stride;
} pdv_sg_out;

int pdv_spectrogram(struct pdv_ctx* ctx, const pdv_params* p, const pdv_sg_params* sg, pdv_sg_out* out);

/*
 * Beat synthesis alone (eq. 3 with the reference amplitude 1/2), for lists
 * the caller provides.  Frame k's entries are [offsets[k], offsets[k+1]) of
 * w (float), v (double, apparent velocity, m/s) and phase_u32 (phase in
 * units of 2^-32 cycles); its samples are [floor(k N/F), floor((k+1) N/F)).
 * offsets: host [n_frames + 1], offsets[0] = 0, non-decreasing; w, v,
 * phase_u32: host [offsets[n_frames]], weights >= 0; signal: host
 * [n_samples].  1 <= n_frames <= 65535, 1 <= n_samples.  The samples are FP32
 * sums in a fixed order that depends only on the frames, the largest frame's
 * entry count and n_samples (bitwise reproducible).  Device memory beyond the
 * entries and the record is bounded (at most 16 MiB of partial records).
 * Errors: PDV_EINVAL (bad sizes, offsets or weights), PDV_ESTATE (serving),
 * PDV_ENOMEM, PDV_EDEVICE.
 */
int pdv_beat_synthesize(struct pdv_ctx* ctx, int32_t n_frames, const uint64_t* offsets,
                        const float* w, const double* v, const uint32_t* phase_u32,
                        double wavelength, double fs, int32_t n_samples, float* signal);

/*
 * Beat synthesis that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc).  Same operation as pdv_beat_synthesize (eq. 3),
 * with every array in device memory of the context's device: offsets
 * [n_frames + 1] (uint64, non-decreasing), w [offsets[n_frames]] (float,
 * >= 0; a negative weight gives NaN samples), v (double, m/s), phase_u32,
 * and the output signal [n_samples] (float).  The arrays are read as given
 * (not validated).  max_frame_entries: the largest entry count of any frame;
 * with the exact value the record equals pdv_beat_synthesize's bit for bit,
 * another value changes only how the entries are split among blocks (FP32
 * summation order), never which entries are summed.
 * Partial records live in a static per-device array of 16 MiB
 * (2^22 floats) set up when the context is created;
 * the work split never needs more (a longer record is summed without
 * partials).  The work is enqueued on the context's stream and the call
 * returns without waiting: the record is complete once that stream reaches
 * this point.  Every call on one device shares its scratch, so calls that
 * overlap on one device (two streams, two contexts) race; calls in one
 * stream's order do not.
 * Errors: PDV_EINVAL (sizes out of range, host or foreign pointers),
 * PDV_ESTATE (serving, or a context without a device), PDV_EDEVICE.
 */
int pdv_beat_synthesize_static(struct pdv_ctx* ctx, int32_t n_frames, const uint64_t* offsets,
                               const float* w, const double* v, const uint32_t* phase_u32,
                               uint64_t max_frame_entries, double wavelength, double fs, int32_t n_samples,
                               float* signal);

/*
 * STFT magnitude alone: periodic Hann window of nfft (power of two) samples
 * every hop samples over signal[n_samples]; map: host [n_windows x (nfft/2+1)].
 * Returns the window count in *n_windows.
 */
int pdv_stft(struct pdv_ctx* ctx, const float* signal, int32_t n_samples, int32_t nfft, int32_t hop,
             float* map, int32_t* n_windows);

/*
 * Autotuner for pdv_spectrum_batch launches.  Times every candidate launch
 * shape (block size 256/512/1024; persistent grid of 1, 2, 4 or 8 blocks per
 * CU, or one block per item; work items of 2^12 .. 2^18 packets) on the given
 * sets, `repeats` times each, and keeps the fastest (median) as the
 * context's default for later batches.  Every candidate must reproduce the
 * first candidate's tallies bitwise (integer tallies do not depend on the
 * launch shape); a mismatch returns PDV_EDEVICE.  best and report are
 * nullable.
 */
typedef struct pdv_tune_report {
    int32_t candidates;          /* launch shapes timed */
    int32_t invariant;           /* 1 if all candidates gave bitwise-equal tallies */
    double best_ms, worst_ms, default_ms;   /* median transport-kernel times */
} pdv_tune_report;

int pdv_autotune(struct pdv_ctx* ctx, const pdv_params* sets, int32_t n, int32_t repeats,
                 pdv_launch_opts* best, pdv_tune_report* report);
/* Set the context's default launch shape (e.g. from a cached tuning). */
int pdv_set_launch_defaults(struct pdv_ctx* ctx, const pdv_launch_opts* opts);
/* Identifier of the kernel sources the library was built from. */
const char* pdv_build_id(void);

/*
 * ---------------------------------------------------------------------------
 * Serving: continuous batching of spectrum requests on one device.
 *
 * After pdv_serve_start, clients submit requests from any thread; one
 * scheduler thread owned by the context admits them in arrival order while
 * a request slot and enough of the memory budget are free, builds their
 * device tables once, and transports a slice of every active request's
 * packets in each persistent launch, so requests that arrive while others
 * run share the device with them.  Results are bitwise the same as a lone
 * pdv_spectrum call with the same parameters (integer tallies over the same
 * random streams).  While a context serves, pdv_spectrum, pdv_spectrum_batch,
 * pdv_spectrogram, pdv_beat_synthesize and pdv_stft return PDV_ESTATE.
 * ---------------------------------------------------------------------------
 */
enum { PDV_EXEC_HIP = 0, PDV_EXEC_HOST = 1 };

typedef struct pdv_serve_opts {
    int32_t max_active;            /* request slots (0 = 256, at most 4096) */
    int32_t max_items;             /* work items per launch (0 = 8192) */
    uint64_t mem_budget;           /* device bytes for active requests (0 = half the context budget) */
    uint64_t packets_per_iteration;/* packets shared among active requests per launch (0 = 2^25) */
    uint64_t packets_per_item;     /* packets per work item (0 = 2^16) */
    int32_t max_layers;            /* largest n_layers served (0 = 1024) */
    int32_t max_angles;            /* largest n_angles served (0 = 2048) */
    int32_t max_bins;              /* largest n_bins served (0 = 1024) */
    int32_t precision;             /* PDV_FP32 or PDV_FP64 for every request */
    int32_t use_graph;             /* 1: replay each launch from a captured hipGraph */
    int32_t executor;              /* PDV_EXEC_HIP, or PDV_EXEC_HOST: scheduler only, no device work
                                      (every packet is tallied as undetected with unit weight) */
    int32_t host_fail_iteration;   /* PDV_EXEC_HOST: report a device failure at this iteration (0 = never) */
    double host_ns_per_packet;     /* PDV_EXEC_HOST: simulated cost per packet */
    double watchdog_ms;            /* > 0: a launch (with its result copies) still running after this long
                                      fails every active and waiting request with PDV_EDEVICE, and the
                                      context is poisoned (the device may still be busy); 0 = no limit */
    int32_t sg_workers;            /* spectrogram workers, each with its own context and stream (0 = 3, at
                                      most 8); requests with a spectrogram are finished by the next free one */
} pdv_serve_opts;

/*
 * A request: the parameter set (copied at submission, including its density
 * and phase arrays), the caller-owned output (w_fx, w2_fx must stay valid
 * until pdv_poll reports a final status), and optionally a spectrogram
 * (sg and sg_out non-NULL; HIP executor only) computed after the spectrum.
 */
typedef struct pdv_request {
    pdv_params params;
    const pdv_sg_params* sg;
    pdv_spectrum_out* out;
    pdv_sg_out* sg_out;
} pdv_request;

typedef struct pdv_serve_stats {
    uint64_t submitted, completed, failed, cancelled;
    uint64_t iterations;           /* persistent launches issued */
    uint64_t packets, events;      /* of completed requests (events = collisions + surface hits) */
    uint64_t admission_waits;      /* requests that had to wait for a slot or memory */
    uint64_t mem_in_use;           /* bytes held by active requests */
    uint32_t active, pending;
    double p50_ms, p99_ms, mean_ms, max_ms;   /* latency: submission -> result on the host */
    double busy_s;                 /* scheduler time spent in table builds and launches */
    double wall_s;                 /* since pdv_serve_start */
    double prepare_s, launch_s, collect_s;   /* scheduler time per phase: tables, launch + wait, result copies */
    double spectrogram_s;          /* spectrogram worker time */
    double queue_p50_ms;           /* median time from submission to admission */
} pdv_serve_stats;

/* Start the scheduler thread (opts nullable).  PDV_ESTATE if already serving. */
int pdv_serve_start(struct pdv_ctx* ctx, const pdv_serve_opts* opts);
/* Queue a request; *ticket identifies it.  Thread-safe.  PDV_EINVAL (bad
 * parameters, beyond the serving limits, or PDV_FLAG_DEVICE_OUTPUT: served
 * results are host arrays), PDV_ENOMEM (larger than the
 * whole memory budget), PDV_ESTATE (not serving or stopping).  PDV_FLAG_PEEL
 * requests are rejected (PDV_EINVAL). */
int pdv_submit(struct pdv_ctx* ctx, const pdv_request* req, uint64_t* ticket);
/* Status of a request: PDV_PENDING, or its final status (PDV_OK, PDV_EOVERFLOW,
 * PDV_ECANCELLED, PDV_EDEVICE, ...).  wait_ms > 0 waits up to that long,
 * < 0 waits until final.  A final status is reported once; the ticket is
 * then forgotten (PDV_ENOTFOUND afterwards).  Thread-safe. */
int pdv_poll(struct pdv_ctx* ctx, uint64_t ticket, int32_t wait_ms);
/* Cancel a request that has not finished (it ends with PDV_ECANCELLED). */
int pdv_cancel(struct pdv_ctx* ctx, uint64_t ticket);
int pdv_serve_report(struct pdv_ctx* ctx, pdv_serve_stats* stats);
/* Stop serving: drain != 0 finishes queued requests first, else cancels
 * them.  Returns PDV_EDEVICE if the executor failed while serving. */
int pdv_serve_stop(struct pdv_ctx* ctx, int32_t drain);

/* A context without a device, usable only for serving with PDV_EXEC_HOST
 * (scheduler tests on machines without a GPU). */
int pdv_create_host(struct pdv_ctx** out);

/*
 * Timing of the last transport launch on ctx: kernel time between HIP events
 * recorded on the context stream around the launch (ms), grid and block
 * size, number of work items, staged guide bits and LDS bytes per block.
 * Any pointer may be NULL.
 */
int pdv_last_launch(const struct pdv_ctx* ctx, float* kernel_ms, int32_t* grid, int32_t* block,
                    int32_t* n_items, int32_t* guide_bits, int32_t* lds_bytes);
/*
 * Kernel kind of the last transport launch: -1 the generic kernel (reads
 * each set's kind), 1 the FP32 kernel for tabulated or Mie laws on layered
 * clouds, 2 the FP32 kernel for Henyey-Greenstein laws on uniform slabs
 * (both with the paper's surface law, implicit capture and no class
 * tallies).  A launch runs a specialised kernel when all its sets share
 * that kind; every kernel gives the same tallies.  -1 for a NULL ctx.
 */
int pdv_last_launch_kind(const struct pdv_ctx* ctx);

/*
 * ---------------------------------------------------------------------------
 * Peak analysis (Sec. III.C, eq. 31, 34-35).
 *
 * The paper reads the ejecta's velocity-profile coefficient beta and optical
 * thickness tau0 off the main peak of a PDV spectrum: smooth the spectrum by
 * a Fourier low-pass filter, take its peak position x = v_peak / v_fs and the
 * relative curvature I''/I there (second derivative in x), and invert
 * x = 1 + ln(tau0)/beta and I''/I = -beta^2.
 *
 * Each of n_spectra histograms (n_bins equal bins on [v_lo, v_hi), any
 * non-negative scale) is replaced by its DFT modes k = 0..keep_modes
 * (keep_modes < n_bins/2), i.e. the band-limited series
 *   S(t) = (1/n)[A_0 + 2 sum_k (A_k cos(2 pi k t/n) + B_k sin(2 pi k t/n))],
 * t the continuous bin coordinate (t = b at the centre of bin b).  The peak
 * is the maximum of S near the bin with the largest S inside the window
 * search_lo <= v < search_hi (bin centres); it is located with Newton steps
 * on S' within one bin of that bin.
 * ---------------------------------------------------------------------------
 */
typedef struct pdv_peak_params {
    double v_lo, v_hi;           /* histogram range (m/s) */
    int32_t n_bins;              /* 16..4096 */
    int32_t keep_modes;          /* 0 <= keep_modes < n_bins / 2 */
    double v_fs;                 /* free-surface velocity (> 0) */
    double search_lo, search_hi; /* peak window on the bin centres (m/s); must hold a bin centre */
} pdv_peak_params;

typedef struct pdv_peak_result {
    int32_t bin;                 /* bin with the largest smoothed value in the window */
    int32_t status;              /* 0, or 1 if the curvature at the peak is not negative (beta, tau0 NaN) */
    double t_peak;               /* peak position in bins (bin centres at integers) */
    double v_peak, x_peak;       /* peak velocity, and v_peak / v_fs */
    double value;                /* smoothed spectrum at the peak */
    double rel_curvature;        /* I''/I at the peak, derivative in v / v_fs */
    double beta, tau0;           /* sqrt(-rel_curvature), exp(beta (x_peak - 1)) */
} pdv_peak_result;

/*
 * spectra: host array, n_spectra x n_bins, row-major (read during the call).
 * smoothed: nullable host array of the same shape for S at the bin centres.
 * out: host array of n_spectra results.  FP64 throughout.  Errors:
 * PDV_EINVAL (NULL pointers, sizes or window out of range), PDV_ENOMEM,
 * PDV_EDEVICE.
 */
int pdv_peak_analysis(struct pdv_ctx* ctx, const double* spectra, int32_t n_spectra, const pdv_peak_params* params,
                      double* smoothed, pdv_peak_result* out);

/*
 * ---------------------------------------------------------------------------
 * Ejecta front end (Sec. II.B eq. 8-10, Sec. II.C eq. 20-21, Sec. III.B
 * eq. 25-27): a cloud stated by the paper's ejecta parameters.
 *
 * The extinction of the whole ejecta is the exponent of eq. 10,
 *   tau_full = 3 m0 <d^2 Q_ext> / (2 rho0 <d^3>),
 * with number-weighted averages over the log-normal size law (eq. 21)
 * truncated to [d_min, d_max] on the Gauss-Legendre nodes in ln d of the
 * Mie tables, Q_ext from Mie theory (eq. 12).  The slab [v_fs, v_top] holds
 * the share 1 - exp(-beta (v_top/v_fs - 1)) of the exponential mass profile
 * (eq. 20) and that share of the extinction (tau_total).  The SS model's
 * optical thickness (eq. 27) uses K*_ext = g_back Q_ext (eq. 25).
 * ---------------------------------------------------------------------------
 */
typedef struct pdv_ejecta {
    double area_mass;            /* m0, total area mass of the ejecta (kg/m^2), > 0 */
    double density;              /* rho0, particle material density (kg/m^3), > 0 */
    double beta;                 /* velocity-profile coefficient (eq. 20), > 0 */
    double v_fs;                 /* free-surface velocity (m/s), > 0 */
    double v_top;                /* top of the slab (m/s), > v_fs */
    double d_median, sigma_ln, d_min, d_max;   /* size law (m), as in pdv_params */
    int32_t n_size_nodes;        /* Gauss-Legendre nodes, 8..1024 */
    int32_t pad;
    double m_re, m_im;           /* complex refractive index (m_im >= 0) */
    double wavelength;           /* m */
    double g_back;               /* K*_ext / K_ext for tau0_ss (0.5-0.7 in the paper; 0 allowed) */
} pdv_ejecta;

typedef struct pdv_ejecta_out {
    double tau_full;             /* extinction optical depth of the whole ejecta (eq. 10) */
    double tau_total;            /* ... of the slab [v_fs, v_top] */
    double mass_share;           /* mass share of the slab */
    double albedo;               /* <C_sca>/<C_ext> (eq. 11) */
    double q_ext_mean;           /* <d^2 Q_ext>/<d^2> */
    double d_sauter;             /* <d^3>/<d^2> (m) */
    double tau0_ss;              /* eq. 27 with K*_ext = g_back Q_ext */
} pdv_ejecta_out;

/*
 * Fill the cloud fields of *p (kept: detector, histogram, packets, seed,
 * precision, surface albedo and law, n_layers, n_angles, max_orders,
 * weighting): v_bottom = v_surface = v_fs, v_top, density EXP with
 * v0 = v_fs/beta, tau_total, phase MIE with the size law and optics.
 * Builds (or reuses) the device Mie tables of that optics; *out (nullable)
 * receives the quantities above.  Errors: PDV_EINVAL (bad ejecta or
 * template), PDV_ENOMEM, PDV_EDEVICE.
 */
int pdv_ejecta_params(struct pdv_ctx* ctx, const pdv_ejecta* ejecta, pdv_params* p, pdv_ejecta_out* out);

#ifdef __cplusplus
}
#endif

#endif /* PDV_H */
