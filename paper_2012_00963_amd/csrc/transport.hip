// Photon-packet transport and tally kernel (gfx950).
//
// Implements the Monte Carlo procedure of Shi et al., Sec. II.B, with exact
// free-flight sampling through layers of constant extinction:
//   free flight      s = -ln u (Beer-Lambert, eq. 7-8), depth change -s mu;
//   surface          diffuse reflection off the moving free surface (the text
//                    after eq. 18; Lambert as an option), weight x surface albedo;
//   particle hit     scatter with probability K_sca/K_ext (eq. 11): implicit
//                    capture multiplies the weight, analog mode draws;
//                    polar angle from the phase function (eq. 13-14, or
//                    Henyey-Greenstein), uniform azimuth (eq. 15), vertical
//                    direction cosine from the third line of eq. 16;
//   Doppler          each scattering off a scatterer of speed V moving along
//                    the normal adds V (mu_out - mu_in)/2 to the apparent
//                    velocity (eq. 4 in velocity units), kept as two
//                    non-negative accumulators so the FP32 difference does
//                    not cancel near the surface peak;
//   exit             photons leaving the top inside the detector cone are
//                    histogrammed by apparent velocity (eq. 19).
// Every event draws one Philox4x32-10 block with counter (k, pid lo, pid hi,
// stream): word 0 the flight, word 1 the polar angle / surface angle, word 2
// the azimuth, word 3 the analog absorption test.
//
// Execution shape: one packet per lane.  A block stages one parameter set's
// tables (layer depths + uniform-depth guide, integer phase CDF + guide; in
// FP32 each depth and CDF entry beside the inverse width of its layer or
// cell) and
// a private histogram in LDS; the histogram carries the velocity bins and
// one slot per terminal sink, so every finished packet costs one LDS atomic
// (two for a binned detection).  A finished lane keeps its packet's final
// state until enough lanes of its wave have finished; the wave then tallies
// them together and refills them from a wave-private range of the work item
// (one LDS atomic per range), so the divergent tally and refill code runs
// once per round instead of on nearly every event.  Table searches are bisections inside the window of a guide of
// up to 2^14 cells (the launch picks the finest that fits its LDS budget);
// the guides are fine enough that most windows hold one entry, and a
// wave leaves the search as soon as all of its lanes have converged.  Event counters and absorbed
// weight live in registers, are reduced across the wave and reach global
// memory with one atomic per wave; the LDS histogram is flushed with global
// 64-bit atomics when the block changes set or retires.  Tallies are
// integers (weight x 2^32), so results do not depend on the launch shape.
#include <algorithm>
#include <map>
#include <mutex>

#include "pdv_device.h"
#include "pdv_internal.h"

namespace pdv {

struct LdsLayout {
    uint32_t t_off, lg_off, cdf_off, cg_off, hist_off, hist2_off, peel_off, peel2_off, und_off, list_off, bytes;
};

// A guide cell's margin (in finest cells) around the scaled depth: covers
// the FP32 rounding of t x scale and of the FP32 layer depths against the
// FP64 depths the guide was built from (both below 2^-8 of a cell).
constexpr float GUIDE_MARGIN = 1.0f / 32.0f;

// Henyey-Greenstein asymmetries below this magnitude take the expanded,
// cancellation-free inversion in FP32 (hg_angle)
constexpr double HG_SMALL_G = 0.1;

__host__ __device__ inline uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }

// terminal-sink slots follow the velocity bins in the LDS histogram
constexpr int N_SINK_SLOTS = 8;

// lane states of the event loop
enum LaneState : int { ST_EMPTY = 0, ST_ALIVE = 1, ST_EXIT = 2, ST_TRUNC = 3, ST_ABS_SURF = 4, ST_ABS_PART = 5 };

// packet indices a wave claims from its work item at a time (fewer for a
// small item, so that every wave of the block gets some)
constexpr int REFILL_CHUNK = 128;
constexpr int REFILL_CHUNK_MIN = 32;

// Detected-list staging: each wave of a list-writing launch gathers up to
// LIST_STAGE entries in LDS and appends them to the frame's list with one
// global atomic, instead of one per retire round.
constexpr int LIST_STAGE = 64;

__host__ __device__ inline LdsLayout lds_layout(int real_bytes, int max_layers, int max_cells, int max_bins,
                                                int guide_bits, int list_waves, bool peel, int threads) {
    const uint32_t guide_entries = (1u << guide_bits) + 1u;
    LdsLayout L;
    // FP32 launches stage each layer depth and CDF entry beside the inverse
    // width of its layer or cell (8-byte entries); FP64 launches stage the
    // plain tables
    const uint32_t t_entry = 8u, c_entry = real_bytes == 4 ? 8u : 4u;
    L.t_off = 0;
    L.lg_off = align16(L.t_off + t_entry * (uint32_t)(max_layers + 1));
    L.cdf_off = align16(L.lg_off + 2u * guide_entries);
    L.cg_off = align16(L.cdf_off + c_entry * (uint32_t)(max_cells + 1));
    L.hist_off = align16(L.cg_off + 2u * guide_entries);
    L.hist2_off = align16(L.hist_off + 8u * (uint32_t)(max_bins + N_SINK_SLOTS));
    // next-event launches: sum(c) and sum(c^2) per bin (their scores outside
    // the bin range go to two of the sink slots)
    L.peel_off = align16(L.hist2_off + 8u * (uint32_t)max_bins);
    L.peel2_off = align16(L.peel_off + (peel ? 8u * (uint32_t)max_bins : 0u));
    // undetected exits: one 64-bit slot per thread, which only that thread
    // adds to (nearly every packet ends there; one shared slot serialised
    // the wave's atomics on a single address)
    L.und_off = align16(L.peel2_off + (peel ? 8u * (uint32_t)max_bins : 0u));
    L.list_off = align16(L.und_off + 8u * (uint32_t)threads);
    L.bytes = align16(L.list_off + (uint32_t)sizeof(ListEntry) * LIST_STAGE * (uint32_t)list_waves);
    return L;
}

template <typename Real>
struct SetConst {            // wave-uniform per-set constants (kept in SGPRs)
    Real tau, v_top, dzeta, zeta_per_tau, v_surface, surface_albedo, albedo, cos_cone;
    Real hg_a, hg_b, hg_c0, hg_c1, hg_inv2g, hg_g;
    Real lg_scale, rev_per_cell, dtheta;
    Real alpha, sin_cone, sin2_cone, peel_surface_m, cells_per_rad;
    double v_lo, dv, inv_dv;
    uint32_t k0, k1, stream, thr_albedo, thr_surface, flags;
    int n_layers, n_cells, n_bins, max_orders, phase_kind, surface_law, weighting;
    int albedo_one, surface_one, hg_zero, hg_small, uniform_density;
};

template <typename Real>
__device__ __forceinline__ SetConst<Real> load_const(const SetDesc& d) {
    SetConst<Real> c;
    c.tau = (Real)d.tau_total;
    c.v_top = (Real)d.v_top;
    c.dzeta = (Real)d.dzeta;
    c.zeta_per_tau = (Real)d.zeta_per_tau;
    c.v_surface = (Real)d.v_surface;
    if constexpr (sizeof(Real) == 4) {
        c.surface_albedo = d.surface_albedo_f;
        c.albedo = d.albedo_f;
    } else {
        c.surface_albedo = d.surface_albedo;
        c.albedo = d.albedo;
    }
    c.cos_cone = (Real)d.cos_cone;
    c.hg_a = (Real)d.hg_a;
    c.hg_b = (Real)d.hg_b;
    c.hg_c0 = (Real)d.hg_c0;
    c.hg_c1 = (Real)d.hg_c1;
    c.hg_inv2g = (Real)d.hg_inv2g;
    c.hg_g = (Real)d.hg_g;
    c.hg_zero = d.hg_g == 0.0;
    c.hg_small = d.hg_g > -HG_SMALL_G && d.hg_g < HG_SMALL_G;
    c.lg_scale = (Real)d.lg_scale;
    c.rev_per_cell = (Real)d.rev_per_cell;
    c.dtheta = (Real)d.dtheta;
    c.alpha = (Real)d.alpha;
    c.sin_cone = (Real)d.sin_cone;
    c.sin2_cone = (Real)d.sin2_cone;
    c.peel_surface_m = (Real)d.peel_surface_m;
    c.cells_per_rad = (Real)d.cells_per_rad;
    c.v_lo = d.v_lo;
    c.dv = d.dv;
    c.inv_dv = d.inv_dv;
    c.k0 = (uint32_t)(d.seed & 0xffffffffu);
    c.k1 = (uint32_t)(d.seed >> 32);
    c.stream = d.stream;
    c.thr_albedo = d.thr_albedo;
    c.thr_surface = d.thr_surface;
    c.flags = d.flags;
    c.n_layers = d.n_layers;
    c.n_cells = d.n_cells;
    c.n_bins = d.n_bins;
    c.max_orders = d.max_orders;
    c.phase_kind = d.phase_kind;
    c.surface_law = d.surface_law;
    c.weighting = d.weighting;
    c.albedo_one = d.albedo_one;
    c.surface_one = d.surface_one;
    c.uniform_density = d.uniform_density;
    return c;
}

// Tests of the set's kind: read from the set (KIND < 0) or fixed at compile
// time for a launch whose sets all share the kind.
template <int KIND>
struct Kind {
    template <typename C> static __device__ __forceinline__ bool table(const C& c) {
        if constexpr (KIND < 0) return c.phase_kind == PH_TABLE; else return (KIND & KB_TABLE) != 0;
    }
    template <typename C> static __device__ __forceinline__ bool uniform(const C& c) {
        if constexpr (KIND < 0) return c.uniform_density != 0; else return (KIND & KB_UNIFORM) != 0;
    }
    template <typename C> static __device__ __forceinline__ bool lambert(const C& c) {
        if constexpr (KIND < 0) return c.surface_law == 1; else return (KIND & KB_LAMBERT) != 0;
    }
    template <typename C> static __device__ __forceinline__ bool analog(const C& c) {
        if constexpr (KIND < 0) return c.weighting == 1; else return (KIND & KB_ANALOG) != 0;
    }
    template <typename C> static __device__ __forceinline__ bool cls(const C& c) {
        if constexpr (KIND < 0) return (c.flags & SF_CLASS) != 0; else return (KIND & KB_CLASS) != 0;
    }
};

// Staged table entries: FP32 launches pair each layer depth T[j] with
// 1/(T[j+1] - T[j]) and each CDF entry C[j] with 1/(C[j+1] - C[j]), so the
// interpolation inside the found layer or cell reads one entry and
// multiplies instead of dividing; FP64 launches divide, as the oracle does.
template <typename Real> struct Staged;
template <> struct Staged<float> {
    using TE = float2;
    using CE = uint2;
};
template <> struct Staged<double> {
    using TE = double;
    using CE = uint32_t;
};
__device__ __forceinline__ float key_of(const float2& e) { return e.x; }
__device__ __forceinline__ double key_of(const double& e) { return e; }
__device__ __forceinline__ uint32_t key_of(const uint2& e) { return e.x; }
__device__ __forceinline__ uint32_t key_of(const uint32_t& e) { return e; }

// Velocity coordinate at depth t.  Uniform density: zeta is linear in depth.
// Otherwise the layer j with T[j] <= t < T[j+1] lies between the guide
// entries of the cells just below and just above t x scale (padded by
// GUIDE_MARGIN); the staged guide keeps every 2^gshift-th cell, so the
// lower cell index rounds down and the upper one up.  zeta is linear inside
// the layer.
template <typename Real>
struct Window {
    int lo, hi;
};

// The guide window of the layer holding depth t (guide reads only).
template <typename Real>
__device__ __forceinline__ Window<Real> zeta_window(const SetConst<Real>& c, const uint16_t* lg, int gshift, Real t) {
    const Real x = t * c.lg_scale;
    int a = (int)(x - (Real)GUIDE_MARGIN);
    int b = (int)(x + (Real)GUIDE_MARGIN) + 1;
    a = a < 0 ? 0 : (a > LAYER_GUIDE - 1 ? LAYER_GUIDE - 1 : a);
    b = b < 0 ? 0 : (b > LAYER_GUIDE ? LAYER_GUIDE : b);    // depths outside the slab stay in bounds
    Window<Real> w;
    w.lo = lg[a >> gshift];
    w.hi = lg[(b + (1 << gshift) - 1) >> gshift];
    return w;
}

// Bisection inside the window until every lane of the wave has converged,
// then the velocity coordinate, linear inside the layer.
template <typename Real>
__device__ __forceinline__ Real zeta_finish(const SetConst<Real>& c, const typename Staged<Real>::TE* T,
                                            Window<Real> w, Real t) {
    int lo = w.lo, hi = w.hi > c.n_layers - 1 ? c.n_layers - 1 : w.hi;
    while (__ballot(lo < hi) != 0ull) {
        const int mid = (lo + hi + 1) >> 1;
        const bool le = key_of(T[mid]) <= t;
        lo = le ? mid : lo;
        hi = le ? hi : mid - 1;
    }
    Real frac;
    if constexpr (sizeof(Real) == 4) {
        const float2 e = T[lo];
        frac = (t - e.x) * e.y;
    } else {
        frac = M<Real>::div(t - T[lo], T[lo + 1] - T[lo]);
    }
    return M<Real>::fma(-((Real)lo + frac), c.dzeta, c.v_top);
}

template <typename Real, int KIND>
__device__ __forceinline__ Real zeta_at(const SetConst<Real>& c, const typename Staged<Real>::TE* T,
                                        const uint16_t* lg, int gshift, Real t) {
    if (Kind<KIND>::uniform(c)) return M<Real>::fma(-t, c.zeta_per_tau, c.v_top);
    return zeta_finish<Real>(c, T, zeta_window<Real>(c, lg, gshift, t), t);
}

// Scattering angle from the integer CDF: the cell is the last j with
// C[j] <= x; it lies between the guide entries of the top guide_bits bits of
// x; the angle is uniform inside the cell.  Returned in units of the cell
// grid (cell index plus the fraction inside it).
// The cell of a 32-bit CDF value x: the last j with C[j] <= x, between the
// guide entries of the top guide_bits bits of x.
__device__ __forceinline__ Window<float> table_window(const uint16_t* cg, int guide_bits, uint32_t x) {
    const uint32_t gi = x >> (32 - guide_bits);
    Window<float> w;
    w.lo = cg[gi];
    w.hi = cg[gi + 1];
    return w;
}

template <typename CE>
__device__ __forceinline__ int table_search(const CE* C, Window<float> w, uint32_t x) {
    int lo = w.lo, hi = w.hi;
    while (__ballot(lo < hi) != 0ull) {
        const int mid = (lo + hi + 1) >> 1;
        const bool le = key_of(C[mid]) <= x;
        lo = le ? mid : lo;
        hi = le ? hi : mid - 1;
    }
    return lo;
}

template <typename CE>
__device__ __forceinline__ int table_cell_of(const CE* C, const uint16_t* cg, int guide_bits, uint32_t x) {
    return table_search(C, table_window(cg, guide_bits, x), x);
}

// Cell index plus the fraction inside the cell (uniform angle in a cell)
template <typename Real>
__device__ __forceinline__ Real table_frac(const typename Staged<Real>::CE* C, int lo, uint32_t x) {
    if constexpr (sizeof(Real) == 4) {
        const uint2 e = C[lo];
        return (Real)lo + ((Real)(x - e.x) + (Real)0.5) * __uint_as_float(e.y);
    } else {
        // C[n_cells] holds 0, so the last cell's width 2^32 - C[j] comes from
        // the unsigned wrap; a zero difference can only mean one cell holding
        // all mass
        const uint32_t cj = C[lo];
        const uint32_t dw = C[lo + 1] - cj;
        const Real width = dw != 0u ? (Real)dw : (Real)4294967296.0;
        return (Real)lo + M<Real>::div((Real)(x - cj) + (Real)0.5, width);
    }
}

template <typename Real>
__device__ __forceinline__ Real table_cells(const typename Staged<Real>::CE* C, const uint16_t* cg, int guide_bits,
                                            uint32_t x) {
    return table_frac<Real>(C, table_cell_of(C, cg, guide_bits, x), x);
}

// Henyey-Greenstein polar cosine by inversion of its cumulative
// distribution (eq. 13's phase function replaced by the HG law):
//   cos = (1 + g^2 - q^2) / (2g),  q = (1 - g^2) / (1 + g s),  s = 2u - 1.
// Written this way the FP32 numerator cancels to O(g) while its rounding
// stays O(2^-24), so the cosine's error grows as 2^-24/|g| (about 1e-3 at
// g = 1e-4).  Expanding the numerator and dividing out the common factor 2g
// gives the same function without the cancellation,
//   cos = [s + g (s^2 + 3)/2 + g^2 s + g^3 (s^2 - 1)/2] / (1 + g s)^2,
// which the FP32 kernels use for |g| < HG_SMALL_G (exactly 2u - 1 at g = 0);
// beyond it the direct form is the better conditioned one (the expanded
// numerator cancels for back-scattering at large g).  FP64 keeps the direct
// form, whose error 2^-53/|g| stays below 1e-12 for |g| >= 1e-4.

template <typename Real>
__device__ __forceinline__ void hg_angle(const SetConst<Real>& c, Real u, Real& ct, Real& st) {
    Real x;
    if (sizeof(Real) == 4 && c.hg_small) {
        const Real s = M<Real>::fma((Real)2.0, u, (Real)-1.0);       // exact
        const Real t = M<Real>::fma(c.hg_g, s, (Real)1.0);
        const Real s2 = s * s;
        const Real inner = M<Real>::fma((Real)0.5 * c.hg_g, s2 - (Real)1.0, s);
        const Real mid = M<Real>::fma(c.hg_g, inner, M<Real>::fma((Real)0.5, s2, (Real)1.5));
        x = M<Real>::fma(c.hg_g, mid, s) * M<Real>::rcp(t * t);
    } else if (c.hg_zero) {
        x = M<Real>::fma((Real)2.0, u, (Real)-1.0);
    } else {
        const Real q = M<Real>::div(c.hg_b, M<Real>::fma(c.hg_c1, u, c.hg_c0));
        if constexpr (sizeof(Real) == 4) x = M<Real>::fma(-q, q, c.hg_a) * c.hg_inv2g;
        else x = M<Real>::fma(-q, q, c.hg_a) / c.hg_c1;
    }
    x = M<Real>::clamp1(x);
    ct = x;
    const Real s2 = ((Real)1.0 - x) * ((Real)1.0 + x);
    st = M<Real>::sqrt(s2 > (Real)0.0 ? s2 : (Real)0.0);
}

// ---------------------------------------------------------------------------
// Next-event (peel-off) estimate of the detector tally.
//
// A photon leaving a scattering or a reflection at depth T with direction
// cosine mu' > 0 leaves the top without another interaction with
// probability exp(-T/mu') (Beer-Lambert, eq. 7), and the detector (eq. 19)
// takes it if mu' >= cos alpha.  The expected detected weight of the event's
// next flight, w a E[1(mu' >= cos alpha) exp(-T/mu')] (a the event's albedo,
// the expectation over the scattering law of eq. 13-16 or the surface law),
// is scored at the apparent velocity the photon carries after the event
// (eq. 4).  Summed over all events its expectation is the detector tally,
// because every detected photon left its last event that way.  One draw
// restricted to the directions that can reach the cone estimates the
// expectation, with the probability of that set of directions as weight:
//   surface, uniform polar angle: psi uniform on [0, alpha], weight
//     alpha / (pi/2); Lambert: mu'^2 uniform on [cos^2 alpha, 1], weight
//     sin^2 alpha;
//   particle: the cone lies within alpha of the vertical, so the scattering
//     angle lies within alpha of the incoming polar angle theta0 = acos(mu):
//     it is drawn from the law restricted to [max(0, theta0 - alpha),
//     min(pi, theta0 + alpha)] (weight: the law's mass there), then the
//     azimuth uniformly from the arc |phi| <= phi_c on which the new
//     direction is inside the cone, cos phi_c = (cos alpha - mu cos Theta) /
//     (sqrt(1 - mu^2) sin Theta) (weight phi_c / pi).
// Every weight lies in [0, 1].  The draw takes its own Philox block (counter
// word 0 = event index with the top bit set), so the transport's own draws
// are untouched and the ordinary tally is the same with or without it.
// ---------------------------------------------------------------------------

// HG probability of cos Theta <= x, written without cancellation:
// (1 - g)(1 + x) / (r (1 + g + r)), r = sqrt(1 + g^2 - 2 g x); the inverse
// of hg_angle's map from u to cos Theta
template <typename Real>
__device__ __forceinline__ Real hg_cdf(const SetConst<Real>& c, Real x) {
    const Real D = M<Real>::fma(-c.hg_c1, x, c.hg_a);
    const Real r = M<Real>::sqrt(D > (Real)0 ? D : (Real)0);
    const Real den = r * ((Real)1.0 + c.hg_g + r);
    return den > (Real)0 ? M<Real>::div(c.hg_c0 * ((Real)1.0 + x), den) : (Real)1.0;
}

// Width of CDF cell j in units of 2^-32 (the last cell ends at 2^32; a
// zero width is a cell of zero mass)
template <typename CE>
__device__ __forceinline__ uint64_t cell_width(const CE* C, int n_cells, int j) {
    const uint64_t next = j + 1 < n_cells ? (uint64_t)key_of(C[j + 1]) : 4294967296ull;
    return next - (uint64_t)key_of(C[j]);
}

// Tabulated law: probability (units of 2^-32) that the angle lies below the
// angle x cells from 0 (uniform angle inside a cell)
template <typename CE>
__device__ __forceinline__ double table_cdf_at(const CE* C, int n_cells, double x) {
    if (x <= 0.0) return 0.0;
    if (x >= (double)n_cells) return 4294967296.0;
    int j = (int)floor(x);
    j = j > n_cells - 1 ? n_cells - 1 : j;
    return (double)key_of(C[j]) + (x - (double)j) * (double)cell_width(C, n_cells, j);
}

// Weight of one restricted draw after a particle scattering (incoming
// direction cosine mu, sm = sqrt(1 - mu^2), depth T) or a reflection; also
// returns 1 - mu' of the drawn direction.
template <typename Real, int KIND>
__device__ __forceinline__ Real peel_weight(const SetConst<Real>& c, const typename Staged<Real>::CE* C,
                                            const uint16_t* cg, int guide_bits, bool surf, Real mu, Real sm, Real T,
                                            Real ur, Real uphi, Real& omc) {
    constexpr Real PI = (Real)3.14159265358979323846;
    if (surf) {
        Real mu_n, M_;
        if (Kind<KIND>::lambert(c)) {
            const Real t = c.sin2_cone * ((Real)1.0 - ur);
            mu_n = M<Real>::sqrt((Real)1.0 - t);
            omc = M<Real>::div(t, (Real)1.0 + mu_n);
        } else {
            Real sh;
            if constexpr (sizeof(Real) == 4) {
                // half the angle, in revolutions: alpha ur / (4 pi)
                sh = M<Real>::sin_rev(c.alpha * ur * (Real)0.0795774715459476679);
                omc = (Real)2.0 * sh * sh;
                mu_n = (Real)1.0 - omc;
            } else {
                const Real psi = c.alpha * ur;
                sh = ::sin((Real)0.5 * psi);
                mu_n = ::cos(psi);
                omc = (Real)2.0 * sh * sh;
            }
        }
        M_ = c.peel_surface_m;
        return mu_n > (Real)0 ? M_ * M<Real>::exp_neg(M<Real>::div(c.tau, mu_n)) : (Real)0;
    }
    const Real ca = c.cos_cone;
    Real cth, sth, M_;
    if (Kind<KIND>::table(c)) {
        const int nc = c.n_cells;
        const Real theta0 = M<Real>::acos(mu);
        const Real th_lo = theta0 - c.alpha > (Real)0 ? theta0 - c.alpha : (Real)0;
        const Real th_hi = theta0 + c.alpha < PI ? theta0 + c.alpha : PI;
        if constexpr (sizeof(Real) == 8) {
            const double y_lo = table_cdf_at(C, nc, th_lo / c.dtheta);
            const double y_hi = table_cdf_at(C, nc, th_hi / c.dtheta);
            M_ = (y_hi - y_lo) * 2.3283064365386963e-10;
            const double y = y_lo + (y_hi - y_lo) * ur;
            const double yf = floor(y);
            const uint32_t xi = yf >= 4294967295.0 ? 0xffffffffu : (uint32_t)yf;
            const int lo = table_cell_of(C, cg, guide_bits, xi);
            const double width = (double)cell_width(C, nc, lo);
            const double f = width > 0.0 ? (y - (double)C[lo]) / width : 0.0;
            const double th = ((double)lo + f) * c.dtheta;
            cth = ::cos(th);
            sth = ::sin(th);
        } else {
            // the bounds in cell units; the law's mass between them and the
            // drawn offset from the lower cell's start stay in 32-bit
            // integers plus small FP32 parts
            float x_lo = th_lo * c.cells_per_rad, x_hi = th_hi * c.cells_per_rad;
            x_hi = x_hi < (float)nc ? x_hi : (float)nc;
            int jl = (int)x_lo, jh = (int)x_hi;
            jl = jl > nc - 1 ? nc - 1 : jl;
            jh = jh > nc - 1 ? nc - 1 : jh;
            const float fl = x_lo - (float)jl, fh = x_hi - (float)jh;
            const uint32_t cl = C[jl].x, chh = C[jh].x;
            const float m_units = M<float>::fma(fh, (float)cell_width(C, nc, jh),
                                                M<float>::fma(-fl, (float)cell_width(C, nc, jl), (float)(chh - cl)));
            M_ = m_units * 2.3283064365386963e-10f;
            const float o = M<float>::fma(m_units, ur, fl * (float)cell_width(C, nc, jl));
            const float of = floorf(o);
            uint64_t xi = (uint64_t)cl + (uint64_t)(o > 0.f ? of : 0.f);
            xi = xi > 0xffffffffull ? 0xffffffffull : xi;
            const int lo = table_cell_of(C, cg, guide_bits, (uint32_t)xi);
            const uint2 e = C[lo];
            const float cells = (float)lo + ((float)((uint32_t)xi - e.x) + (o - of)) * __uint_as_float(e.y);
            const float rev = cells * c.rev_per_cell;
            cth = M<float>::cos_rev(rev);
            sth = M<float>::sin_rev(rev);
        }
    } else {
        Real u_lo, u_hi;
        if constexpr (sizeof(Real) == 8) {
            const Real theta0 = ::acos(mu);
            const Real th_lo = theta0 - c.alpha > 0.0 ? theta0 - c.alpha : 0.0;
            const Real th_hi = theta0 + c.alpha < PI ? theta0 + c.alpha : PI;
            u_lo = hg_cdf(c, ::cos(th_hi));
            u_hi = hg_cdf(c, ::cos(th_lo));
        } else {
            // cos(theta0 -+ alpha) = mu cos alpha +- sqrt(1 - mu^2) sin alpha,
            // cut at 0 and pi
            const float c_lo = mu >= ca ? 1.0f : M<float>::fma(mu, ca, sm * c.sin_cone);
            const float c_hi = mu <= -ca ? -1.0f : M<float>::fma(mu, ca, -sm * c.sin_cone);
            u_lo = hg_cdf(c, c_hi);
            u_hi = hg_cdf(c, c_lo);
        }
        M_ = u_hi - u_lo;
        hg_angle<Real>(c, M<Real>::fma(M_, ur, u_lo), cth, sth);
    }
    const Real den = sm * sth;
    Real phi_c;
    if (den <= (sizeof(Real) == 4 ? (Real)1e-30 : (Real)1e-300)) {
        phi_c = PI;                      // every azimuth gives mu' = mu cos Theta
    } else {
        const Real kappa = M<Real>::div(ca - mu * cth, den);
        phi_c = kappa <= (Real)-1 ? PI : (kappa >= (Real)1 ? (Real)0 : M<Real>::acos(kappa));
    }
    Real cphi;
    if constexpr (sizeof(Real) == 4) cphi = M<float>::cos_rev(phi_c * uphi * 0.159154943091895336f);
    else cphi = ::cos(phi_c * uphi);
    Real mu_n = M<Real>::fma(mu, cth, den * cphi);
    mu_n = mu_n > (Real)1 ? (Real)1 : mu_n;
    omc = (Real)1.0 - mu_n;
    if (!(M_ > (Real)0) || phi_c <= (Real)0 || mu_n <= (Real)0) return (Real)0;
    Real share;
    if constexpr (sizeof(Real) == 4) share = phi_c * 0.318309886183790672f;
    else share = phi_c / PI;
    return M_ * share * M<Real>::exp_neg(M<Real>::div(T, mu_n));
}

// Event counters: collisions, surface hits and the absorbed weight (fixed
// point) are a lane's running sums over the packets it finished in the
// current set, reduced across the wave when the block changes set or
// finishes.  Packet, exit and detection counts are not kept per lane or per
// wave: the packets of each work item are added when the item is taken, the
// rare outcomes (a detection, a packet that ends inside the cloud) add one
// to a block counter in their own branch, and the exits are the packets
// less those that ended inside, formed at the set's flush.
struct LaneAcc {
    uint64_t abs_particle, abs_surface;
    uint32_t collisions, surface;
};

__device__ __forceinline__ void flush_acc(LaneAcc& a, uint64_t* tally, int n_bins) {
    const uint64_t s_ap = wave_sum_u64(a.abs_particle);
    const uint64_t s_as = wave_sum_u64(a.abs_surface);
    const uint64_t c_c = wave_sum_u64(a.collisions);
    const uint64_t c_s = wave_sum_u64(a.surface);
    if (lane_id() == 0) {
        unsigned long long* sk = (unsigned long long*)(tally + tw_sinks(n_bins));
        if (s_ap) atomicAdd(sk + SK_ABS_PARTICLE, (unsigned long long)s_ap);
        if (s_as) atomicAdd(sk + SK_ABS_SURFACE, (unsigned long long)s_as);
        unsigned long long* ct = (unsigned long long*)(tally + tw_counts(n_bins));
        if (c_c) atomicAdd(ct + C_COLLISIONS, (unsigned long long)c_c);
        if (c_s) atomicAdd(ct + C_SURFACE, (unsigned long long)c_s);
    }
    a = LaneAcc{0, 0, 0, 0};
}

// Occupancy targets: the specialised FP32 kernels fit eight waves per SIMD
// (64 VGPRs, run as two 1024-thread blocks per CU), the generic FP32 kernel
// six, the FP64 kernel four.
template <typename Real, bool LIST, int KIND, bool PEEL>
__global__ void __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 ? (KIND >= 0 && !PEEL ? 8 : 6) : 4, 8)))
transport_kernel(const SetDesc* __restrict__ descs, const uint8_t* __restrict__ tables,
                 uint64_t* __restrict__ tallies, const WorkItem* __restrict__ items, int n_items,
                 uint32_t* __restrict__ queue, int persistent, int max_layers, int max_cells, int max_bins,
                 ListEntry* __restrict__ lists, uint64_t* __restrict__ list_counts,
                 const int* __restrict__ n_items_dev, int guide_bits, int retire_min) {
    extern __shared__ __align__(16) uint8_t lds[];
    // Packets on a uniform slab under the HG law scatter about 1.5 times on
    // average, so a whole round spent on each packet's final flight out of
    // the cloud is a large share of the work: this kind draws and tests every
    // next flight at the end of the event before it (the same blocks, the
    // same arithmetic, the same decisions).  The first flight is drawn when
    // the packet starts, for all packets of a retire round together.
    constexpr bool LOOKAHEAD = KIND == KIND_HG_UNIFORM && !PEEL && sizeof(Real) == 4;
    if (n_items_dev) n_items = *n_items_dev;   // item count from device memory (graph replays)
    __shared__ WorkItem s_item;
    __shared__ int s_item_idx;
    __shared__ uint32_t s_next;
    // the current set's packets taken by this block (added by thread 0 per
    // item, or by each wave for the items it takes itself), how many of them
    // were detected and how many ended inside the cloud
    __shared__ unsigned long long s_packets, s_detected, s_ended;

    const LdsLayout L = lds_layout((int)sizeof(Real), max_layers, max_cells, max_bins, guide_bits,
                                   LIST ? (int)(blockDim.x >> 6) : 0, PEEL, (int)blockDim.x);
    const int gshift = GUIDE_BITS - guide_bits;
    const int n_guide = 1 << guide_bits;
    using TE = typename Staged<Real>::TE;
    using CE = typename Staged<Real>::CE;
    TE* sT = (TE*)(lds + L.t_off);
    uint16_t* sLG = (uint16_t*)(lds + L.lg_off);
    CE* sC = (CE*)(lds + L.cdf_off);
    uint16_t* sCG = (uint16_t*)(lds + L.cg_off);
    unsigned long long* sW = (unsigned long long*)(lds + L.hist_off);     // bins, then sink slots
    unsigned long long* sW2 = (unsigned long long*)(lds + L.hist2_off);
    unsigned long long* sU = (unsigned long long*)(lds + L.und_off);      // this block's threads' undetected weight
    unsigned long long* sP = (unsigned long long*)(lds + L.peel_off);     // next-event sum(c), sum(c^2)
    unsigned long long* sP2 = (unsigned long long*)(lds + L.peel2_off);

    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = lane_id();
    // this wave's list staging (list-writing launches) and its fill, which
    // is wave-uniform
    ListEntry* sL = (ListEntry*)(lds + L.list_off) + (uint32_t)(tid >> 6) * LIST_STAGE;
    uint32_t l_fill = 0;
    // append the staged entries to set's list: one atomic reserves the slots,
    // lane i copies entry i (entries past the list's capacity are counted,
    // not stored)
    // Staged entries hold the packet id's low word in place of the phase
    // word; the flush forms each entry's phase word (the packet's Philox
    // block with event counter 0xFFFFFFFF), one lane per entry, so the block
    // is drawn once per staged detection instead of by the whole wave in
    // every retire round that has one.  pid_hi: the high word of every
    // packet id of the current work item (items do not cross a multiple of
    // 2^32).
    auto flush_list = [&](int set, uint32_t pid_hi) {
        if (l_fill == 0) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const SetDesc& d = descs[set];
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long*)(list_counts + set), (unsigned long long)l_fill);
        base = __shfl(base, 0, 64);
        if ((uint32_t)lane < l_fill) {
            ListEntry e = sL[lane];
            const uint32_t k0 = (uint32_t)(d.seed & 0xffffffffu), k1 = (uint32_t)(d.seed >> 32);
            uint32_t p0, p1;
            philox_packet_words(e.phase, pid_hi, k0, p0, p1);
            e.phase = philox10_event(0xffffffffu, p0, p1, d.stream ^ k1, k0, k1).x;
            const unsigned long long slot = base + (unsigned long long)lane;
            if (slot < d.list_capacity) lists[d.list_offset + slot] = e;
        }
        __builtin_amdgcn_wave_barrier();
        l_fill = 0;
    };
    int cur_set = -1;
    LaneAcc acc = LaneAcc{0, 0, 0, 0};
    if (tid == 0) {
        s_packets = 0ull;
        s_detected = 0ull;
        s_ended = 0ull;
    }

    auto flush_set = [&](int set) {
        const SetDesc& d = descs[set];
        uint64_t* tally = tallies + d.tally_offset;
        flush_acc(acc, tally, d.n_bins);
        __syncthreads();
        if (tid == 0) {
            unsigned long long* ct = (unsigned long long*)(tally + tw_counts(d.n_bins));
            if (s_packets) atomicAdd(ct + C_PACKETS, s_packets);
            if (s_packets - s_ended) atomicAdd(ct + C_EXITS, s_packets - s_ended);
            if (s_detected) atomicAdd(ct + C_DETECTED, s_detected);
            s_packets = 0ull;
            s_detected = 0ull;
            s_ended = 0ull;
        }
        unsigned long long* gW = (unsigned long long*)(tally + tw_w(d.n_bins));
        unsigned long long* gW2 = (unsigned long long*)(tally + tw_w2(d.n_bins));
        unsigned long long* gS = (unsigned long long*)(tally + tw_sinks(d.n_bins));
        for (int b = tid; b < d.n_bins; b += nthr) {
            const unsigned long long w = sW[b], w2 = sW2[b];
            if (w) atomicAdd(gW + b, w);
            if (w2) atomicAdd(gW2 + b, w2);
        }
        if constexpr (PEEL) {
            if (d.flags & SF_PEEL) {
                unsigned long long* gP = (unsigned long long*)(tally + tw_peel(d.n_bins, d.flags));
                unsigned long long* gP2 = (unsigned long long*)(tally + tw_peel2(d.n_bins, d.flags));
                for (int b = tid; b < d.n_bins; b += nthr) {
                    const unsigned long long v = sP[b], v2 = sP2[b];
                    if (v) atomicAdd(gP + b, v);
                    if (v2) atomicAdd(gP2 + b, v2);
                }
            }
        }
        if (tid < N_SINK_SLOTS) {
            const unsigned long long v = sW[d.n_bins + tid];
            if (v) atomicAdd(gS + tid, v);
        }
        {
            // the threads' undetected weight: summed per wave, one atomic each
            const unsigned long long u = wave_sum_u64(sU[tid]);
            if (lane == 0 && u) atomicAdd(gS + SK_UNDETECTED, u);
        }
        __syncthreads();
    };

    // persistent == 2 (one set, no lists): the block stages the set of item 0
    // once and every wave then takes work items from the launch's queue by
    // itself, whenever its packet range runs out, without waiting for its
    // lanes to finish the packets they hold; the block meets only when the
    // queue is empty.  Otherwise the block takes items one at a time and
    // shares each among its waves.
    // (list-writing launches keep block items: a wave's staged entries share
    // one high packet-id word, that of the item they came from)
    const bool wave_items = persistent == 2 && !LIST;
    for (int it = 0;; ++it) {
        if (tid == 0) {
            int idx = wave_items ? (it == 0 ? 0 : n_items)
                                 : (persistent ? (int)atomicAdd(queue, 1u) : (it == 0 ? (int)blockIdx.x : n_items));
            s_item_idx = idx;
            if (idx < n_items) s_item = items[idx];
            s_next = 0;
        }
        __syncthreads();
        const int idx = (int)uniform_u32((uint32_t)s_item_idx);
        if (idx >= n_items) break;
        const int set = (int)uniform_u32(s_item.set);
        uint64_t pid0 = s_item.pid_begin;          // the current item's first packet id (per wave with wave_items)
        const uint32_t count = (uint32_t)s_item.count;
        // wave_items: item 0 holds the whole set, cut into n_items equal
        // items (sizes differ by one at most, larger ones first)
        const uint64_t set_pid = s_item.pid_begin;
        uint64_t wi_even = 0, wi_extra = 0;
        if (wave_items) {
            wi_even = s_item.count / (uint64_t)n_items;
            wi_extra = s_item.count % (uint64_t)n_items;
        }

        if (set != cur_set) {
            if (cur_set >= 0) flush_set(cur_set);
            const SetDesc& d = descs[set];
            const uint8_t* tb = tables + d.tab_offset;
            if (!d.uniform_density) {
                const double* gT64 = (const double*)(tb + TableLayout::T64);
                if constexpr (sizeof(Real) == 4) {
                    // the inverse widths come from the FP64 depths (an empty
                    // layer, which no search returns, gets 0)
                    const float* gT = (const float*)(tb + TableLayout::T32);
                    for (int i = tid; i <= d.n_layers; i += nthr) {
                        const double w = i < d.n_layers ? gT64[i + 1] - gT64[i] : 0.0;
                        sT[i] = make_float2(gT[i], w > 0.0 ? (float)(1.0 / w) : 0.0f);
                    }
                } else {
                    for (int i = tid; i <= d.n_layers; i += nthr) sT[i] = gT64[i];
                }
                const uint16_t* gLG = (const uint16_t*)(tb + TableLayout::LGUIDE);
                for (int i = tid; i <= n_guide; i += nthr) sLG[i] = gLG[i << gshift];
            }
            if (d.phase_kind == PH_TABLE) {
                const uint32_t* gC = (const uint32_t*)(tb + TableLayout::CDF);
                if constexpr (sizeof(Real) == 4) {
                    // a cell's width is the next entry minus its own; the last
                    // cell ends at 2^32 (a zero width can only mean one cell
                    // holding all mass)
                    for (int i = tid; i < d.n_cells; i += nthr) {
                        const uint32_t cj = gC[i];
                        const uint32_t dw = (i + 1 < d.n_cells ? gC[i + 1] : 0u) - cj;
                        const double width = dw != 0u ? (double)dw : 4294967296.0;
                        sC[i] = make_uint2(cj, __float_as_uint((float)(1.0 / width)));
                    }
                    if (tid == 0) sC[d.n_cells] = make_uint2(0u, 0u);
                } else {
                    for (int i = tid; i < d.n_cells; i += nthr) sC[i] = gC[i];
                    if (tid == 0) sC[d.n_cells] = 0u;
                }
                const uint16_t* gCG = (const uint16_t*)(tb + TableLayout::CGUIDE);
                for (int i = tid; i <= n_guide; i += nthr) sCG[i] = gCG[i << gshift];
            }
            for (int i = tid; i < d.n_bins + N_SINK_SLOTS; i += nthr) sW[i] = 0ull;
            for (int i = tid; i < d.n_bins; i += nthr) sW2[i] = 0ull;
            sU[tid] = 0ull;
            if constexpr (PEEL) {
                for (int i = tid; i < d.n_bins; i += nthr) {
                    sP[i] = 0ull;
                    sP2[i] = 0ull;
                }
            }
            cur_set = set;
            __syncthreads();
        }

        // read by thread 0 at the set's flush (with wave_items the waves add
        // the items they take)
        if (tid == 0 && !wave_items) s_packets += count;
        const SetConst<Real> c = load_const<Real>(descs[set]);
        const int nb = c.n_bins;
        uint32_t chunk = count / (2u * (uint32_t)(nthr >> 6));
        chunk = chunk < (uint32_t)REFILL_CHUNK_MIN ? (uint32_t)REFILL_CHUNK_MIN
                                                   : (chunk > (uint32_t)REFILL_CHUNK ? (uint32_t)REFILL_CHUNK : chunk);

        // ---- per-lane packet state ----
        // st: ST_EMPTY (no packet), ST_ALIVE, or how the packet ended (its
        // tally waits for the wave's next retire round)
        int st = ST_EMPTY;
        bool exhausted = false;              // the item has no packets left for this wave
        uint32_t w_next = 0, w_end = 0;      // wave-private range of item-local packet indices
        bool first_item = true;              // with wave_items: the wave has not taken an item yet
        uint64_t pid = 0;
        uint32_t q0 = 0, q1 = 0;             // the packet's fixed first-round Philox words
        uint32_t k = 0;
        int n_sc = 0, n_surf = 0;
        Real T = 0, mu = -1, w = 1, big = 0, small = 0, abs_s = 0;
        // look-ahead kinds: the next flight's depth and the block words the
        // next event uses, drawn at the end of the previous event
        uint32_t cy = 0, cz = 0;
        Real Tc = 0;
        // draws the packet's next Philox block into X_ and returns the
        // optical depth the flight from T_ along mu_ reaches (eq. 10: the
        // path length in optical depth is -ln u)
        auto draw_flight = [&](Real mu_, Real T_, Block4& X_) -> Real {
            // the key enters opaquely each event, so the ten round keys are
            // recomputed on the scalar unit rather than held in 20 SGPRs
            uint32_t key0 = c.k0, key1 = c.k1;
            asm volatile("" : "+s"(key0), "+s"(key1));
            X_ = philox10_event(k, q0, q1, c.stream ^ key1, key0, key1);
            k += 1;
            return M<Real>::fma(-M<Real>::neg_log(unit_open<Real>(X_.x)), mu_, T_);
        };

        while (true) {
            // Retire and refill in rounds: when retire_min lanes wait (or all
            // do), tally the finished packets and start new ones from the
            // wave's range, claiming a new range from the item when it runs out.
            const uint64_t idle = __ballot(st != ST_ALIVE);
            if (idle == ~0ull || (!exhausted && (int)__popcll(idle) >= retire_min)) {
                bool det_now = false;        // this lane's packet goes to the detected list
                float e_w = 0.f;
                uint32_t e_phase = 0;
                double e_v = 0.0;
                if (st >= ST_EXIT) {
                    // ---- the packet's tally: one terminal slot of the LDS histogram ----
                    const bool detected = st == ST_EXIT && mu >= c.cos_cone;
                    int slot;
                    double vt = 0.0;
                    if (detected) {
                        vt = (double)big - (double)small;
                        double bf;
                        if constexpr (sizeof(Real) == 8) bf = floor((vt - c.v_lo) / c.dv);
                        else bf = floor((vt - c.v_lo) * c.inv_dv);
                        slot = bf < 0.0 ? nb + SK_UNDER : (bf >= (double)nb ? nb + SK_OVER : (int)bf);
                        atomicAdd(&s_detected, 1ull);
                    } else if (st == ST_EXIT) {
                        slot = nb + SK_UNDETECTED;
                    } else {
                        slot = nb + (st == ST_TRUNC ? SK_TRUNCATED
                                                    : (st == ST_ABS_SURF ? SK_ABS_SURFACE : SK_ABS_PARTICLE));
                        atomicAdd(&s_ended, 1ull);
                    }
                    const uint64_t fw = to_fixed32<Real>(w);
                    if (slot == nb + SK_UNDETECTED) sU[tid] += (unsigned long long)fw;
                    else atomicAdd(&sW[slot], (unsigned long long)fw);
                    if (slot < nb) {
                        atomicAdd(&sW2[slot], (unsigned long long)to_fixed32<Real>(w * w));
                        if (Kind<KIND>::cls(c)) {
                            unsigned long long* gcl =
                                (unsigned long long*)(tallies + descs[set].tally_offset + tw_class(nb));
                            if (n_sc == 1 && n_surf == 0) atomicAdd(gcl + slot, (unsigned long long)fw);
                            if (n_sc == 0 && n_surf == 1) atomicAdd(gcl + nb + slot, (unsigned long long)fw);
                        }
                    }
                    if constexpr (LIST) {
                        if (detected) {
                            det_now = true;
                            e_w = (float)w;
                            e_phase = (uint32_t)pid;       // the phase word is formed at the flush
                            e_v = vt;
                        }
                    }
                    // implicit capture: the packet's 2^32 units are split exactly
                    // between its terminal slot and the two absorption sinks
                    if (!Kind<KIND>::analog(c)) {
                        const uint64_t fs = to_fixed32<Real>(abs_s);
                        acc.abs_surface += fs;
                        acc.abs_particle += (4294967296ull - fw) - fs;
                    }
                    acc.collisions += (uint32_t)n_sc;
                    acc.surface += (uint32_t)n_surf;
                    st = ST_EMPTY;
                }
                if constexpr (LIST) {
                    // stage this round's detections (the wave's whole set of
                    // lanes takes part, so the staging fill stays uniform)
                    const uint64_t dm = __ballot(det_now);
                    if (dm != 0ull) {
                        const uint32_t n_new = (uint32_t)__popcll(dm);
                        if (l_fill + n_new > (uint32_t)LIST_STAGE) flush_list(set, (uint32_t)(pid0 >> 32));
                        if (det_now) {
                            const uint32_t r = __builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(dm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)dm, 0u));
                            ListEntry e;
                            e.w = e_w;
                            e.phase = e_phase;
                            e.v = e_v;
                            sL[l_fill + r] = e;
                        }
                        l_fill += n_new;
                    }
                }
                uint64_t empty = __ballot(st == ST_EMPTY);
                while (empty != 0ull && !exhausted) {
                    if (w_next >= w_end) {
                        if (wave_items) {
                            // this wave's next work item (all of the launch's
                            // items belong to the block's one set): its first
                            // one is item (global wave index), so the waves do
                            // not all meet at the queue when the launch starts;
                            // later ones come from the queue, after the first
                            // items of all waves
                            uint32_t qi = 0;
                            if (first_item) {
                                qi = blockIdx.x * (uint32_t)(nthr >> 6) + (uint32_t)(tid >> 6);
                                first_item = false;
                            } else {
                                if (lane == 0) qi = atomicAdd(queue, 1u);
                                qi = uniform_u32(qi) + gridDim.x * (uint32_t)(nthr >> 6);
                            }
                            qi = uniform_u32(qi);
                            if (qi >= (uint32_t)n_items) {
                                exhausted = true;
                                break;
                            }
                            const uint64_t q64 = qi;
                            pid0 = set_pid + q64 * wi_even + (q64 < wi_extra ? q64 : wi_extra);
                            w_next = 0;
                            w_end = (uint32_t)(wi_even + (q64 < wi_extra ? 1u : 0u));
                            if (lane == 0) atomicAdd(&s_packets, (unsigned long long)w_end);
                        } else {
                            uint32_t base = 0;
                            if (lane == 0) base = atomicAdd(&s_next, chunk);
                            base = uniform_u32(base);
                            if (base >= count) {
                                exhausted = true;
                                break;
                            }
                            w_next = base;
                            w_end = count - base < chunk ? count : base + chunk;
                        }
                    }
                    const uint32_t n = (uint32_t)__popcll(empty);
                    const uint32_t avail = w_end - w_next;
                    const uint32_t take = n < avail ? n : avail;
                    if (st == ST_EMPTY) {
                        const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(empty >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)empty, 0u));
                        if (rank < take) {
                            st = ST_ALIVE;
                            pid = pid0 + w_next + rank;
                            philox_packet_words((uint32_t)pid, (uint32_t)(pid >> 32), c.k0, q0, q1);
                            k = 0; n_sc = 0; n_surf = 0;
                            T = 0; mu = -1; w = 1; big = 0; small = 0; abs_s = 0;
                        }
                    }
                    w_next += take;
                    empty = __ballot(st == ST_EMPTY);
                }
                if constexpr (LOOKAHEAD) {
                    // the first flight of each packet started in this round
                    // (downward from the top: it never leaves)
                    if (st == ST_ALIVE && k == 0u) {
                        Block4 Y;
                        Tc = draw_flight(mu, T, Y);
                        cy = Y.y;
                        cz = Y.z;
                    }
                }
                if (__ballot(st == ST_ALIVE) == 0ull) break;
            }
            if (st == ST_ALIVE) {
            Block4 X;
            Real Tn;
            bool leave;
            if constexpr (LOOKAHEAD) {
                // the flight was drawn when the previous event ended (or at the
                // packet's start) and stays inside the cloud
                X = Block4{0u, cy, cz, 0u};
                Tn = Tc;
                leave = false;
            } else {
                Tn = draw_flight(mu, T, X);
                leave = mu > (Real)0 && Tn <= (Real)0;
            }
            const Real u1 = unit_open<Real>(X.y);
            const Real u2 = unit_open<Real>(X.z);
            const bool surf = mu < (Real)0 && Tn >= c.tau;
            const bool coll = !leave && !surf;

            // particle interaction: scatterer speed, scattering angle
            Real Vc = 0, cells = 0, ct = 0, st_ = 0;
            if (coll) {
                Vc = zeta_at<Real, KIND>(c, sT, sLG, gshift, Tn);
                if (Kind<KIND>::table(c)) cells = table_cells<Real>(sC, sCG, guide_bits, X.y);
                else hg_angle<Real>(c, u1, ct, st_);
            }
            // free-surface reflection (computed for every lane, selected below)
            Real mu_s, omc_s;
            if constexpr (sizeof(Real) == 4) {
                // under the paper's surface law a lane needs one sine either
                // way: of the scattering angle if it collides, of half the
                // reflection angle if it reaches the surface
                const bool paper_law = !Kind<KIND>::lambert(c);
                Real sh = 0;
                if (Kind<KIND>::table(c)) {
                    const Real rev = cells * c.rev_per_cell;
                    const Real sv = M<Real>::sin_rev(paper_law && surf ? (Real)0.125 * u1 : rev);
                    ct = M<Real>::cos_rev(rev);
                    st_ = sv;
                    sh = sv;
                } else if (paper_law) {
                    sh = M<Real>::sin_rev((Real)0.125 * u1);
                }
                if (paper_law) {
                    // cos(psi) = 1 - 2 sin^2(psi/2)
                    omc_s = (Real)2.0 * sh * sh;
                    mu_s = (Real)1.0 - omc_s;
                } else {
                    const Real r = M<Real>::sqrt(u1);
                    mu_s = r;
                    omc_s = M<Real>::div((Real)1.0 - u1, (Real)1.0 + r);
                }
            } else {
                if (Kind<KIND>::table(c)) {
                    const Real theta = cells * c.dtheta;
                    ct = ::cos(theta);
                    st_ = ::sin(theta);
                }
                if (Kind<KIND>::lambert(c)) {
                    const Real r = M<Real>::sqrt(u1);
                    mu_s = r;
                    omc_s = M<Real>::div((Real)1.0 - u1, (Real)1.0 + r);
                } else {
                    const Real psi = (Real)0.5 * M<Real>::PI * u1;
                    const Real sh = ::sin((Real)0.5 * psi);
                    mu_s = ::cos(psi);
                    omc_s = (Real)2.0 * sh * sh;
                }
            }
            // new direction of a colliding lane (eq. 16)
            const Real cphi = M<Real>::cos_rev(u2);
            const Real sm2 = ((Real)1.0 - mu) * ((Real)1.0 + mu);
            const Real mu_c = M<Real>::clamp1(
                M<Real>::fma(mu, ct, M<Real>::sqrt(sm2 > (Real)0 ? sm2 : (Real)0) * st_ * cphi));
            const Real omc_c = (Real)1.0 - mu_c;
            const Real V = surf ? c.v_surface : Vc;
            const Real mu_new = surf ? mu_s : mu_c;
            const Real omc = surf ? omc_s : omc_c;
            const Real a = surf ? c.surface_albedo : c.albedo;

            const bool trunc = coll && n_sc == c.max_orders;
            bool absorbed = false;
            if (Kind<KIND>::analog(c)) {
                const uint32_t thr = surf ? c.thr_surface : c.thr_albedo;
                const bool one = surf ? (bool)c.surface_one : (bool)c.albedo_one;
                absorbed = !leave && !trunc && !one && X.w >= thr;
            }
            // next-event estimate of this scattering or reflection, from the
            // state before the event's updates
            if constexpr (PEEL) {
                if ((c.flags & SF_PEEL) && (surf || (coll && !trunc))) {
                    uint32_t key0 = c.k0, key1 = c.k1;
                    asm volatile("" : "+s"(key0), "+s"(key1));
                    const Block4 Q = philox10_event((k - 1u) | 0x80000000u, q0, q1, c.stream ^ key1, key0, key1);
                    const Real sm = M<Real>::sqrt(sm2 > (Real)0 ? sm2 : (Real)0);
                    Real omc_p;
                    const Real wt = peel_weight<Real, KIND>(c, sC, sCG, guide_bits, surf, mu, sm, Tn,
                                                            unit_open<Real>(Q.x), unit_open<Real>(Q.y), omc_p);
                    const Real sc = w * a * wt;
                    const uint64_t fc = to_fixed32<Real>(sc);
                    if (fc != 0ull) {
                        const Real big_p = M<Real>::fma((Real)0.5 * V, (Real)1.0 - mu, big);
                        const Real small_p = M<Real>::fma((Real)0.5 * V, omc_p, small);
                        const double vp = (double)big_p - (double)small_p;
                        double bf;
                        if constexpr (sizeof(Real) == 8) bf = floor((vp - c.v_lo) / c.dv);
                        else bf = floor((vp - c.v_lo) * c.inv_dv);
                        if (bf < 0.0) {
                            atomicAdd(&sW[nb + SK_PEEL_UNDER], (unsigned long long)fc);
                        } else if (bf >= (double)nb) {
                            atomicAdd(&sW[nb + SK_PEEL_OVER], (unsigned long long)fc);
                        } else {
                            const int b = (int)bf;
                            atomicAdd(&sP[b], (unsigned long long)fc);
                            const uint64_t fc2 = to_fixed32<Real>(sc * sc);
                            if (fc2 != 0ull) atomicAdd(&sP2[b], (unsigned long long)fc2);
                        }
                    }
                }
            }
            // the event counts as a collision or surface hit whether or not
            // the packet continues
            n_surf += surf ? 1 : 0;
            n_sc += coll ? 1 : 0;
            if (!(leave || trunc || absorbed)) {
                if (!Kind<KIND>::analog(c)) {
                    const Real lost = w * ((Real)1.0 - a);
                    abs_s += surf ? lost : (Real)0;
                    w *= a;
                }
                big = M<Real>::fma((Real)0.5 * V, (Real)1.0 - mu, big);
                small = M<Real>::fma((Real)0.5 * V, omc, small);
                mu = mu_new;
                T = surf ? c.tau : Tn;
                if constexpr (LOOKAHEAD) {
                    // the next flight now: a packet that leaves the cloud ends
                    // in this round instead of spending another on the flight
                    Block4 Y;
                    Tc = draw_flight(mu, T, Y);
                    cy = Y.y;
                    cz = Y.z;
                    if (mu > (Real)0 && Tc <= (Real)0) st = ST_EXIT;
                }
            } else {
                st = leave ? ST_EXIT : (trunc ? ST_TRUNC : (surf ? ST_ABS_SURF : ST_ABS_PART));
            }
            }  // alive
        }
        // the item's staged detections go out before the next item (which
        // may belong to another set)
        if constexpr (LIST) flush_list(set, (uint32_t)(pid0 >> 32));
        __syncthreads();
    }
    if (cur_set >= 0) flush_set(cur_set);
}

}  // namespace pdv

// ---- host launchers ----
//
// This file is compiled twice.  The default pass builds the FP32 kernels
// without implicit floating-point contraction (every kind of FP32 kernel then
// performs the same roundings) together with the host dispatch; the pass with
// PDV_TRANSPORT_FP64 builds the FP64 kernels, which only exist in the generic
// kind, with the compiler's usual contraction.
namespace pdv {

template <typename Real, bool LIST, int KIND, bool PEEL>
static const void* kernel_ptr() {
    return reinterpret_cast<const void*>(&transport_kernel<Real, LIST, KIND, PEEL>);
}

template <typename Real, bool LIST, int KIND, bool PEEL>
static hipError_t launch_kind(hipStream_t s, const TransportShape& sh, const SetDesc* descs, const uint8_t* tables,
                              uint64_t* tallies, const WorkItem* items, int n_items, const int* n_items_dev,
                              uint32_t* queue, int persistent, ListEntry* lists, uint64_t* list_counts) {
    hipLaunchKernelGGL((transport_kernel<Real, LIST, KIND, PEEL>), dim3(sh.grid), dim3(sh.block), sh.lds_bytes, s,
                       descs, tables, tallies, items, n_items, queue, persistent, sh.max_layers, sh.max_cells,
                       sh.max_bins, lists, list_counts, n_items_dev, sh.guide_bits, sh.retire_min);
    return hipGetLastError();
}

// Kernels of one precision and kind: with or without detected lists, with
// or without the next-event estimate (lists and the estimate are not
// combined).
template <typename Real, int KIND>
static const void* kind_ptr(bool list, bool peel) {
    if (list) return kernel_ptr<Real, true, KIND, false>();
    return peel ? kernel_ptr<Real, false, KIND, true>() : kernel_ptr<Real, false, KIND, false>();
}

template <typename Real, int KIND>
static hipError_t launch_of_kind(hipStream_t s, bool list, const TransportShape& sh, const SetDesc* descs,
                                 const uint8_t* tables, uint64_t* tallies, const WorkItem* items, int n_items,
                                 const int* n_items_dev, uint32_t* queue, int persistent, ListEntry* lists,
                                 uint64_t* list_counts) {
    if (list)
        return launch_kind<Real, true, KIND, false>(s, sh, descs, tables, tallies, items, n_items, n_items_dev, queue,
                                                    persistent, lists, list_counts);
    if (sh.peel)
        return launch_kind<Real, false, KIND, true>(s, sh, descs, tables, tallies, items, n_items, n_items_dev,
                                                    queue, persistent, lists, list_counts);
    return launch_kind<Real, false, KIND, false>(s, sh, descs, tables, tallies, items, n_items, n_items_dev, queue,
                                                 persistent, lists, list_counts);
}

#if defined(PDV_TRANSPORT_FP64)

const void* select_kernel_fp64(bool list, bool peel) { return kind_ptr<double, KIND_GENERIC>(list, peel); }

hipError_t launch_transport_fp64(hipStream_t s, bool list, const TransportShape& sh, const SetDesc* descs,
                                 const uint8_t* tables, uint64_t* tallies, const WorkItem* items, int n_items,
                                 const int* n_items_dev, uint32_t* queue, int persistent, ListEntry* lists,
                                 uint64_t* list_counts) {
    return launch_of_kind<double, KIND_GENERIC>(s, list, sh, descs, tables, tallies, items, n_items, n_items_dev,
                                                queue, persistent, lists, list_counts);
}

#else

// FP64 kernels (the other compilation pass)
const void* select_kernel_fp64(bool list, bool peel);
hipError_t launch_transport_fp64(hipStream_t s, bool list, const TransportShape& sh, const SetDesc* descs,
                                 const uint8_t* tables, uint64_t* tallies, const WorkItem* items, int n_items,
                                 const int* n_items_dev, uint32_t* queue, int persistent, ListEntry* lists,
                                 uint64_t* list_counts);

// FP32 launches of one specialised kind get their own kernel; FP64 (the
// plain baseline) always runs the generic one.
static const void* select_kernel(int precision, bool list, int kind, bool peel) {
    if (precision == 1) return select_kernel_fp64(list, peel);
    if (kind == KIND_TABLE_LAYERED) return kind_ptr<float, KIND_TABLE_LAYERED>(list, peel);
    if (kind == KIND_HG_UNIFORM) return kind_ptr<float, KIND_HG_UNIFORM>(list, peel);
    return kind_ptr<float, KIND_GENERIC>(list, peel);
}

// Per-kernel launch facts, set once: the dynamic LDS a kernel is allowed
// (the attribute call is repeated only for a larger size: each call made the
// next launch on the stream take ~0.2 ms of host time) and its resident
// blocks per CU at a block size.
namespace {
std::mutex g_kmu;
std::map<const void*, int> g_allowed_lds;
std::map<std::pair<const void*, int>, int> g_resident;
}  // namespace

static hipError_t allow_lds(const void* k, int bytes) {
    // dynamic LDS beyond 64 KiB must be allowed per kernel
    if (bytes <= 65536) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_kmu);
    int& cur = g_allowed_lds[k];
    if (cur >= bytes) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) cur = bytes;
    return e;
}

static hipError_t resident_blocks(const void* k, int block, int* resident) {
    std::lock_guard<std::mutex> lk(g_kmu);
    auto it = g_resident.find({k, block});
    if (it != g_resident.end()) {
        *resident = it->second;
        return hipSuccess;
    }
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(resident, k, block, 0);
    if (e == hipSuccess) g_resident[{k, block}] = *resident;
    return e;
}

// Pick the guide resolution and LDS size of a launch and allow that LDS
// size for the kernel (outside any graph capture).  want_bits in
// [MIN_GUIDE_BITS, GUIDE_BITS] forces the resolution; 0 takes the finest
// whose staging lets as many blocks share a CU's LDS as the kernel's
// registers allow.  Fails with hipErrorInvalidValue when even the coarsest
// guide exceeds the per-block LDS limit, or when a next-event launch asks
// for detected lists.
hipError_t plan_transport(TransportShape& sh, int precision, bool list, int want_bits, int lds_per_block,
                          int lds_per_cu) {
    if (list && sh.peel) return hipErrorInvalidValue;
    const int rb = precision == 1 ? 8 : 4;
    const void* kp = select_kernel(precision, list, sh.kind, sh.peel);
    auto bytes = [&](int bits) {
        return (int)lds_layout(rb, sh.max_layers, sh.max_cells, sh.max_bins, bits, list ? sh.block / 64 : 0, sh.peel,
                               sh.block)
            .bytes;
    };
    if (want_bits != 0) {
        if (want_bits < MIN_GUIDE_BITS || want_bits > GUIDE_BITS) return hipErrorInvalidValue;
        sh.guide_bits = want_bits;
    } else {
        int resident = 1;
        hipError_t e = resident_blocks(kp, sh.block, &resident);
        if (e != hipSuccess) return e;
        if (resident < 1) resident = 1;
        const int budget = std::min(lds_per_block, lds_per_cu / resident);
        sh.guide_bits = MIN_GUIDE_BITS;
        for (int b = GUIDE_BITS; b > MIN_GUIDE_BITS; --b)
            if (bytes(b) <= budget) { sh.guide_bits = b; break; }
    }
    sh.lds_bytes = bytes(sh.guide_bits);
    if (sh.lds_bytes > lds_per_block) return hipErrorInvalidValue;
    return allow_lds(kp, sh.lds_bytes);
}

static hipError_t launch_fp32(hipStream_t s, bool list, const TransportShape& sh, const SetDesc* descs,
                              const uint8_t* tables, uint64_t* tallies, const WorkItem* items, int n_items,
                              const int* n_items_dev, uint32_t* queue, int persistent, ListEntry* lists,
                              uint64_t* list_counts) {
    if (sh.kind == KIND_TABLE_LAYERED)
        return launch_of_kind<float, KIND_TABLE_LAYERED>(s, list, sh, descs, tables, tallies, items, n_items,
                                                         n_items_dev, queue, persistent, lists, list_counts);
    if (sh.kind == KIND_HG_UNIFORM)
        return launch_of_kind<float, KIND_HG_UNIFORM>(s, list, sh, descs, tables, tallies, items, n_items,
                                                      n_items_dev, queue, persistent, lists, list_counts);
    return launch_of_kind<float, KIND_GENERIC>(s, list, sh, descs, tables, tallies, items, n_items, n_items_dev,
                                               queue, persistent, lists, list_counts);
}

// Persistent launch whose item count is read from device memory, so a
// captured graph can be replayed with a different item list.
hipError_t launch_transport_dev(hipStream_t s, int precision, const TransportShape& sh, const SetDesc* descs,
                                const uint8_t* tables, uint64_t* tallies, const WorkItem* items,
                                const int* n_items_dev, uint32_t* queue) {
    if (precision == 1)
        return launch_transport_fp64(s, false, sh, descs, tables, tallies, items, 0, n_items_dev, queue, 1, nullptr,
                                     nullptr);
    return launch_fp32(s, false, sh, descs, tables, tallies, items, 0, n_items_dev, queue, 1, nullptr, nullptr);
}

// n_items_dev (nullable): read the item count from device memory instead of
// n_items, so a captured graph can be replayed for another item list.
hipError_t launch_transport(hipStream_t s, int precision, bool list, const TransportShape& sh,
                            const SetDesc* descs, const uint8_t* tables, uint64_t* tallies, const WorkItem* items,
                            int n_items, const int* n_items_dev, uint32_t* queue, int persistent, ListEntry* lists,
                            uint64_t* list_counts) {
    if (precision == 1)
        return launch_transport_fp64(s, list, sh, descs, tables, tallies, items, n_items, n_items_dev, queue,
                                     persistent, lists, list_counts);
    return launch_fp32(s, list, sh, descs, tables, tallies, items, n_items, n_items_dev, queue, persistent, lists,
                       list_counts);
}

#endif  // PDV_TRANSPORT_FP64

}  // namespace pdv
