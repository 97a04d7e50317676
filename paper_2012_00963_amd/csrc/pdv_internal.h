// Internal layout shared by the host side of libpdv and its HIP kernels.
//
// Device memory of a batch (all owned by the context, see pdv_api.cpp):
//   SetDesc[n_sets]      per-set constants (host-packed, finished on device)
//   table arena          per-set tables, SET_TABLE_BYTES each, 256-B aligned
//   tally arena          per-set uint64 tallies, tally_words(n_bins) each
//   WorkItem[n_items]    (set, first packet, packet count), largest set first
//   queue counter        next work item for persistent blocks
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdv {

// Table geometry limits (LDS staging is sized from them per launch).
constexpr int MAX_LAYERS = 4096;
constexpr int MAX_ANGLES = 4096;
// Search guides are stored at 2^GUIDE_BITS cells (+1 entry); a launch stages
// every 2^(GUIDE_BITS - b)-th entry in LDS, b in [MIN_GUIDE_BITS, GUIDE_BITS].
constexpr int GUIDE_BITS = 14;
constexpr int MIN_GUIDE_BITS = 11;
constexpr int LAYER_GUIDE = 1 << GUIDE_BITS;   // uniform-depth cells
constexpr int CDF_GUIDE = 1 << GUIDE_BITS;     // cells of the 2^32 CDF range
constexpr int MAX_BINS = 4096;

enum PhaseKind : int32_t { PH_HG = 0, PH_TABLE = 1 };

// Byte offsets inside one set's table block.
struct TableLayout {
    static constexpr uint64_t T32 = 0;                                        // float[MAX_LAYERS+1]
    static constexpr uint64_t T64 = T32 + 4ull * (MAX_LAYERS + 8);            // double[MAX_LAYERS+1]
    static constexpr uint64_t LGUIDE = T64 + 8ull * (MAX_LAYERS + 8);         // uint16[LAYER_GUIDE+1]
    static constexpr uint64_t CDF = LGUIDE + 2ull * (LAYER_GUIDE + 64);       // uint32[MAX_ANGLES]
    static constexpr uint64_t CGUIDE = CDF + 4ull * (MAX_ANGLES + 64);        // uint16[CDF_GUIDE+1]
    static constexpr uint64_t PHASE = CGUIDE + 2ull * (CDF_GUIDE + 64);       // double[MAX_ANGLES] tabulated p(theta)
    static constexpr uint64_t BYTES = (PHASE + 8ull * MAX_ANGLES + 255) & ~255ull;
};

// Tally block of one set, in uint64 words: sum(w) and sum(w^2) per bin,
// eight sink words (the six terminal sinks, then the next-event scores below
// and above the bin range), eight counters; then, for sets that ask for
// them, the two class tallies (SF_CLASS) and the next-event estimate sum(c)
// and sum(c^2) per bin (SF_PEEL).
enum TallyWords : int { TW_SINKS = 8, TW_COUNTS = 8 };
inline __host__ __device__ uint64_t tw_w(int) { return 0; }
inline __host__ __device__ uint64_t tw_w2(int n_bins) { return (uint64_t)n_bins; }
inline __host__ __device__ uint64_t tw_sinks(int n_bins) { return 2ull * n_bins; }
inline __host__ __device__ uint64_t tw_counts(int n_bins) { return 2ull * n_bins + TW_SINKS; }
inline __host__ __device__ uint64_t tw_class(int n_bins) { return 2ull * n_bins + TW_SINKS + TW_COUNTS; }
inline __host__ __device__ uint64_t tw_peel(int n_bins, uint32_t set_flags) {
    return tw_class(n_bins) + ((set_flags & 1u) ? 2ull * n_bins : 0ull);
}
inline __host__ __device__ uint64_t tw_peel2(int n_bins, uint32_t set_flags) {
    return tw_peel(n_bins, set_flags) + (uint64_t)n_bins;
}
inline __host__ __device__ uint64_t tally_words(int n_bins, uint32_t set_flags) {
    return tw_peel(n_bins, set_flags) + ((set_flags & 4u) ? 2ull * n_bins : 0ull);
}

// sink word indices inside the sinks block (match pdv.h; the last two hold
// next-event scores outside the bin range)
enum SinkIdx : int { SK_UNDER = 0, SK_OVER = 1, SK_UNDETECTED = 2, SK_ABS_PARTICLE = 3,
                     SK_ABS_SURFACE = 4, SK_TRUNCATED = 5, SK_PEEL_UNDER = 6, SK_PEEL_OVER = 7 };
enum CountIdx : int { C_PACKETS = 0, C_COLLISIONS = 1, C_SURFACE = 2, C_EXITS = 3, C_DETECTED = 4 };

// Per-set constants.  Host fills everything except the fields marked
// (device), which the table kernels write.
struct alignas(16) SetDesc {
    double v_top, dzeta, tau_total;
    double v_surface, surface_albedo;
    double albedo;              // (device for Mie) single-scattering albedo
    double hg_g;
    double g_mean;              // (device) mean cosine of the sampled law
    double cos_cone;
    double v_lo, dv, inv_dv;
    double zeta_per_tau;        // uniform density: (v_top - v_bottom) / tau_total
    // detector cone for the next-event estimate: half angle alpha (as
    // acos(cos alpha)), sin alpha, sin^2 alpha, the share of reflected
    // directions inside the cone under the set's surface law, and angle
    // cells per radian of the tabulated law
    double alpha, sin_cone, sin2_cone, peel_surface_m, cells_per_rad;
    // precomputed Henyey-Greenstein constants: 1+g^2, 1-g^2, 1-g, 2g, 1/(2g)
    double hg_a, hg_b, hg_c0, hg_c1, hg_inv2g;
    double lg_scale;            // LAYER_GUIDE / tau_total (finest guide cells per unit depth)
    double rev_per_cell;        // 0.5 / n_cells (table angle in revolutions)
    double dtheta;              // pi / n_cells
    uint64_t seed;
    uint64_t tab_offset;        // bytes into the table arena
    uint64_t tally_offset;      // words into the tally arena
    uint64_t list_offset;       // entries into the list arena
    uint64_t list_capacity;
    uint32_t stream;
    uint32_t thr_albedo;        // (device for Mie) floor(albedo 2^32), clamped
    uint32_t thr_surface;
    uint32_t flags;
    int32_t n_layers;
    int32_t phase_kind;         // PH_HG or PH_TABLE
    int32_t n_cells;            // tabulated angles - 1
    int32_t surface_law;
    int32_t weighting;
    int32_t max_orders;
    int32_t n_bins;
    int32_t albedo_one;         // (device for Mie) 1 if albedo >= 1
    int32_t surface_one;
    int32_t uniform_density;    // 1: zeta is linear in depth, no table search
    // the two albedos rounded to FP32 (albedo_f: device for Mie): the FP32
    // kernel selects between them per lane, from scalar registers
    float albedo_f;
    float surface_albedo_f;
};

// One device-to-device copy of tally words into a caller's array.
struct CopyJob {
    uint64_t src_word;          // first word in the tally arena
    uint64_t n_words;
    uint64_t* dst;              // caller's device array
};

struct WorkItem {
    uint32_t set;
    uint32_t pad;
    uint64_t pid_begin;         // absolute packet id of the first packet
    uint64_t count;
};

// Detected-list entry (stage 2): weight, raw phase word, apparent velocity.
struct alignas(16) ListEntry {
    float w;
    uint32_t phase;
    double v;
};

enum SetFlags : uint32_t { SF_CLASS = 1u, SF_LIST = 2u, SF_PEEL = 4u };
static_assert(SF_CLASS == 1u && SF_PEEL == 4u, "tally_words() tests these flag bits");

// Beat synthesis work split: blocks take (sample tile, frame, group of
// entry chunks); the entries of a frame are split into groups only while
// the grid stays below SYNTH_TARGET_BLOCKS and the groups' partial records
// fit SYNTH_PARTIAL_MAX_FLOATS, so the partials never exceed 16 MiB.
constexpr uint64_t SYNTH_TARGET_BLOCKS = 8192;
constexpr uint64_t SYNTH_PARTIAL_MAX_FLOATS = 1ull << 22;
constexpr int SYNTH_MAX_FRAMES = 65535;
struct SynthPlan {
    int max_samples;           // samples of the longest frame, ceil(N / F)
    int tiles;                 // sample tiles of the longest frame
    int n_groups;              // entry-chunk groups per frame (1: no partial records)
    int cpg;                   // chunks per group (the last group takes the rest)
    uint64_t partial_floats;   // partial-record floats the split needs
};

// Set kinds.  A launch whose sets all share one of the specialised kinds
// runs a transport kernel with the kind's tests resolved at compile time
// (fewer branches and scalar registers); any other launch runs the generic
// kernel, which reads them from each set.  Both perform the same arithmetic.
enum KindBits : int { KB_TABLE = 1, KB_UNIFORM = 2, KB_LAMBERT = 4, KB_ANALOG = 8, KB_CLASS = 16 };
constexpr int KIND_GENERIC = -1;
constexpr int KIND_TABLE_LAYERED = KB_TABLE;      // tabulated or Mie law, layered cloud, paper surface law, implicit
constexpr int KIND_HG_UNIFORM = KB_UNIFORM;       // Henyey-Greenstein law, uniform slab, paper surface law, implicit

// Launch shape of the transport kernel (host side).
struct TransportShape {
    int grid = 1, block = 512;
    int max_layers = 0, max_cells = 0, max_bins = 0;   // LDS staging sizes of the batch
    int guide_bits = GUIDE_BITS;                        // staged guide resolution
    int lds_bytes = 0;
    int retire_min = 12;                                // finished lanes per retire round
    int kind = KIND_GENERIC;                            // kernel specialisation (FP32 only)
    bool peel = false;                                  // next-event estimate for sets that ask for it
};

// Peak analysis (host-packed constants of one call) and its per-spectrum result.
struct PeakJob {
    double v_lo, dv, v_fs, search_lo, search_hi;
    int32_t wb0, wb1;          // first and last bin with its centre in the window
};
struct PeakOut {
    int32_t bin, status;
    double t_peak, v_peak, x_peak, value, rel_curvature, beta, tau0;
};

// Ejecta front end: the constants of one call.
struct EjectaJob {
    double area_mass, density, beta, v_fs, v_top, d_median, sigma_ln, g_back;
};

// Table-building jobs (host-packed, one per set).
struct LayerJob {
    double v_bottom, v_top, v0, tau_total;
    int32_t n_layers, density_kind;
    uint64_t tab_offset;
    uint64_t density_offset;   // doubles into the density staging buffer (TABLE kind)
};

struct PhaseJob {
    int32_t kind;              // 0 = Mie basis, 1 = caller table already in PHASE
    int32_t n_angles;
    double d_median, sigma_ln;
    uint64_t tab_offset;
    int32_t set;               // descriptor to finish
    int32_t pad;
};

// One size node of the Mie basis.
struct MieNodeInfo {
    double x;                  // size parameter pi d / lambda
    double lnd;                // ln d
    double wq;                 // Gauss-Legendre weight in ln d
    double q_ext, q_sca, g;
    int32_t nstop;
    int32_t pad;
};

}  // namespace pdv
