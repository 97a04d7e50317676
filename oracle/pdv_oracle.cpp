// PDV multiple-scattering Monte Carlo — FP64 CPU ORACLE.
//
// TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
// cpu_baseline leg of bench.py may load this library.  The product (the HIP
// library under paper_2012_00963_amd/) never calls it and shares no code
// with it.
//
// What it computes (Shi et al., "Reconstruction and interpretation of PDV
// spectrum for ejecta particles", Sec. II):
//   * photons enter the top of a laterally infinite slab of moving particles
//     travelling straight down (Sec. II.B procedure step 1, boundary eq. 6);
//   * free flight obeys Beer-Lambert attenuation (eq. 7-8) through layers of
//     piecewise-constant extinction (Sec. II.B step 2 uses 1000 layers);
//   * at an interaction the photon is scattered with probability K_sca/K_ext
//     and absorbed otherwise (eq. 11); the packet weight carries this
//     probability (implicit capture) or a Bernoulli draw decides (analog);
//   * a scattered photon takes a new polar angle from the phase function
//     (eq. 13-14, or Henyey-Greenstein) and a uniform azimuth (eq. 15); only
//     the vertical direction cosine matters in a 1-D slab with vertical
//     velocities, so it follows the third line of eq. 16;
//   * each scattering changes the frequency by the Doppler term of eq. 4,
//     kept in velocity units: a scatterer of speed V moving along +z shifts
//     the apparent velocity by V*(mu_out - mu_in)/2;
//   * at the free surface the photon is reflected diffusely with polar angle
//     uniform over the upper hemisphere (Sec. II.B, text after eq. 18) or by
//     Lambert's law (option), and the moving surface adds its own shift;
//   * photons leaving the top inside the detector cone are histogrammed by
//     apparent velocity (eq. 19, intensity form).
//
// Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), one 4-word block per
// event: counter = (event k, pid low, pid high, stream), key = seed.
//
// Everything is plain scalar FP64 with no blocking or reordering; threads
// take contiguous packet ranges and their tallies are added in thread order.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

// ---- Philox4x32-10 from its published definition (Salmon et al. 2011) ----
// Round function: two 32x32->64 products of words 0 and 2 with the fixed
// multipliers; the high halves are xored with the other words and the key.
// Between rounds the key is bumped by the Weyl constants (golden ratio and
// sqrt(3)-1 scaled to 32 bits).
const uint32_t PHILOX_M0 = 0xD2511F53u;
const uint32_t PHILOX_M1 = 0xCD9E8D57u;
const uint32_t PHILOX_W0 = 0x9E3779B9u;
const uint32_t PHILOX_W1 = 0xBB67AE85u;

void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// A 32-bit word to a uniform in (0,1): the top 23 bits give an odd multiple
// of 2^-24, exactly representable in binary32 and binary64 alike.
double uniform_from_word(uint32_t x) {
    return (double)(2u * (x >> 9) + 1u) * (1.0 / 16777216.0);
}

const double PI = 3.14159265358979323846;

enum { PHASE_HG = 0, PHASE_TABLE = 1 };
enum { SURFACE_UNIFORM_THETA = 0, SURFACE_LAMBERT = 1 };
enum { WEIGHT_IMPLICIT = 0, WEIGHT_ANALOG = 1 };
enum { SINK_UNDER = 0, SINK_OVER, SINK_UNDETECTED, SINK_ABSORBED_PARTICLE,
       SINK_ABSORBED_SURFACE, SINK_TRUNCATED, N_SINKS };
enum { CNT_PACKETS = 0, CNT_COLLISIONS, CNT_SURFACE, CNT_EXITS, CNT_DETECTED, CNT_FLIGHTS, N_COUNTS };

}  // namespace

extern "C" {

typedef struct {
    /* slab in velocity coordinate zeta = z / t (m/s); particle speed = zeta */
    double v_bottom, v_top;
    int n_layers;
    const double* T;          /* n_layers+1 cumulative extinction depth from the top */
    double tau_total;
    /* phase function */
    int phase_kind;           /* PHASE_HG or PHASE_TABLE */
    double hg_g;
    int n_angles;             /* table grid theta_j = j*pi/(n_angles-1) */
    const uint64_t* cdf;      /* n_angles entries, cdf[0]=0, cdf[n_angles-1]=2^32 */
    double albedo;            /* single-scattering albedo K_sca/K_ext */
    /* free surface */
    double v_surface, surface_albedo;
    int surface_law;
    /* detector and histogram */
    double cos_cone;
    double v_lo, v_hi;
    int n_bins;
    int max_orders;
    int weighting;
    /* packets and random streams */
    uint64_t pid_begin, n_packets;
    uint64_t seed;
    uint32_t stream;
    int n_threads;
    /* 1: also score the next-event (peel-off) estimate of the cone tally */
    int peel;
} oracle_params;

typedef struct {
    double* W;                /* [n_bins] sum of w per velocity bin */
    double* W2;               /* [n_bins] sum of w^2 */
    double* W_single;         /* [n_bins] nullable: one particle scattering, no surface */
    double* W_surface;        /* [n_bins] nullable: no particle scattering, one surface hit */
    double sinks[N_SINKS];
    uint64_t counts[N_COUNTS];
    /* detected list (nullable arrays): weight, apparent velocity, beat phase in cycles, pid */
    uint64_t list_capacity;
    uint64_t list_count;      /* number that would have been written (may exceed capacity) */
    double* list_w;
    double* list_v;
    double* list_phase;
    uint64_t* list_pid;
    /* nullable: first-order bound on how far an FP32 evaluation of the same
     * path (same branch decisions) can move the apparent velocity */
    double* list_err32;
    /* next-event estimate (peel != 0): per bin the sum of the expected
     * direct-exit weights scored at every scattering and reflection, and the
     * sum of their squares; nullable class arrays for scores at a packet's
     * first particle scattering (no surface hit before) and at its first
     * surface hit (no particle scattering before); scores outside the bin
     * range (under, over) */
    double* P;
    double* P2;
    double* P_single;
    double* P_surface;
    double peel_sinks[2];
} oracle_out;

void oracle_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    philox4x32_10(ctr, key, out);
}

}  // extern "C"

namespace {

struct Tally {
    std::vector<double> W, W2, Ws, Wsurf;
    std::vector<double> P, P2, Ps, Psurf;   // next-event estimate (empty if off)
    double peel_sinks[2] = {0};
    double sinks[N_SINKS] = {0};
    uint64_t counts[N_COUNTS] = {0};
    bool keep_list = false;
    std::vector<double> lw, lv, lph, lerr;
    std::vector<uint64_t> lpid;
};

// ---------------------------------------------------------------------------
// First-order rounding bound of an FP32 evaluation of one packet's path.
//
// Carried beside the FP64 path only when detected lists are kept: absolute
// bounds on the FP32 depth (eT), direction cosine (eMu) and the two Doppler
// accumulators (eBig, eSmall), given that every branch decision (flight end,
// cell, exit, cone, bin) comes out the same.  U = 2^-24 is the FP32 unit
// roundoff; each formula adds the inputs' propagated errors (partial
// derivative times input error) and the roundings of the operations, with a
// few U for the hardware transcendental units (log, sin, cos, sqrt, rcp).
// The apparent velocity is the FP64 difference of the two FP32
// accumulators, so its bound is eBig + eSmall.
// ---------------------------------------------------------------------------
struct Fp32Bound {
    static constexpr double U = 5.9604644775390625e-08;   // 2^-24
    double eT = 0.0, eMu = 0.0, eBig = 0.0, eSmall = 0.0;

    // free path s = -ln u0 and the new depth T + s (-mu)
    double flight(double s, double mu, double Tn) const {
        const double es = 4.0 * U * (s + 1.0);
        return eT + std::fabs(mu) * es + s * eMu + U * std::fabs(Tn);
    }
    // accumulator update acc += term with the term's own error e_term
    static double acc(double e_acc, double e_term, double term, double acc_new) {
        return e_acc + e_term + 2.0 * U * std::fabs(term) + U * std::fabs(acc_new);
    }
    // collision at depth Tn (error eTn) in a layer of slope dzeta/dT, new
    // cosine from the polar angle (cosine x, sine sn, their errors ex, es)
    // and the azimuth cosine cphi
    void collision(double eTn, double Tn, double slope, double V, double mu, double x, double sn, double ex,
                   double es, double cphi, double mu_new, double big_new, double small_new) {
        const double eV = slope * (eTn + 2.0 * U * std::fabs(Tn)) + 4.0 * U * std::fabs(V);
        const double r = std::sqrt(std::fmax(0.0, (1.0 - mu) * (1.0 + mu)));
        const double er = std::fabs(mu) * eMu / std::fmax(r, std::sqrt(2.0 * eMu + 2.0 * U)) + 2.0 * U;
        const double ecphi = 4.0 * U;
        const double eMu_new = std::fabs(x) * eMu + std::fabs(mu) * ex + std::fabs(sn * cphi) * er +
                               std::fabs(r * cphi) * es + std::fabs(r * sn) * ecphi + 3.0 * U;
        const double tb = 0.5 * V * (1.0 - mu), ts = 0.5 * V * (1.0 - mu_new);
        eBig = acc(eBig, 0.5 * ((1.0 - mu) * eV + V * (eMu + U)), tb, big_new);
        eSmall = acc(eSmall, 0.5 * ((1.0 - mu_new) * eV + V * (eMu_new + U)), ts, small_new);
        eMu = eMu_new;
        eT = eTn;
    }
    // reflection off the surface at speed vs: new cosine 1 - omc with its
    // complement omc computed directly (error eOmc)
    void surface(double vs, double mu, double omc, double eOmc, double eMu_new, double tau, double big_new,
                 double small_new) {
        const double tb = 0.5 * vs * (1.0 - mu), ts = 0.5 * vs * omc;
        eBig = acc(eBig, 0.5 * vs * (eMu + U), tb, big_new);
        eSmall = acc(eSmall, 0.5 * vs * eOmc, ts, small_new);
        eMu = eMu_new;
        eT = U * tau;                 // the depth is reset to the FP32 slab depth
    }
    // error of a sine formed as sqrt((1 - x)(1 + x)) from a cosine of error ex
    static double sine_err(double x, double sn, double ex) {
        return std::fabs(x) * ex / std::fmax(sn, std::sqrt(2.0 * ex)) + 2.0 * U;
    }
};

// Layer holding depth t, searched by bisection: T[j] <= t < T[j+1].
int find_layer(const oracle_params& p, double t) {
    int lo = 0, hi = p.n_layers - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (p.T[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Velocity coordinate of a collision at depth t: linear inside the layer
// (constant extinction per layer), layer j spanning zeta from
// v_top - j*dzeta down to v_top - (j+1)*dzeta.
double zeta_at_depth(const oracle_params& p, double t) {
    int j = find_layer(p, t);
    double dzeta = (p.v_top - p.v_bottom) / p.n_layers;
    double frac = (t - p.T[j]) / (p.T[j + 1] - p.T[j]);
    return p.v_top - ((double)j + frac) * dzeta;
}

// Cosine and sine of the scattering angle drawn from the tabulated phase
// function: the cell is the last j with cdf[j] <= x (an integer comparison),
// and the angle is uniform inside the cell.
void table_angle(const oracle_params& p, uint32_t x, double* c, double* s) {
    int lo = 0, hi = p.n_angles - 2;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (p.cdf[mid] <= (uint64_t)x) lo = mid; else hi = mid - 1;
    }
    double width = (double)(p.cdf[lo + 1] - p.cdf[lo]);
    double f = ((double)((uint64_t)x - p.cdf[lo]) + 0.5) / width;
    double dtheta = PI / (double)(p.n_angles - 1);
    double theta = ((double)lo + f) * dtheta;
    *c = std::cos(theta);
    *s = std::sin(theta);
}

// Henyey-Greenstein polar cosine by inversion of its cumulative distribution.
void hg_angle(double g, double u, double* c, double* s) {
    double ct;
    if (g == 0.0) {
        ct = 2.0 * u - 1.0;
    } else {
        double q = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
        ct = (1.0 + g * g - q * q) / (2.0 * g);
    }
    if (ct > 1.0) ct = 1.0;
    if (ct < -1.0) ct = -1.0;
    *c = ct;
    double s2 = (1.0 - ct) * (1.0 + ct);
    *s = std::sqrt(s2 > 0.0 ? s2 : 0.0);
}

// New vertical direction cosine after a particle scattering: polar angle
// from the phase function, azimuth uniform (eq. 15), and the third line of the
// direction update (eq. 16), clamped to [-1, 1].
// cth, sth, cphi (nullable) receive the polar angle's cosine and sine and
// the azimuth's cosine.
double scattered_mu(const oracle_params& p, double mu, uint32_t x1, double u1, double u2,
                    double* cth_out = nullptr, double* sth_out = nullptr, double* cphi_out = nullptr) {
    double cth, sth;
    if (p.phase_kind == PHASE_TABLE) table_angle(p, x1, &cth, &sth);
    else hg_angle(p.hg_g, u1, &cth, &sth);
    const double cphi = std::cos(2.0 * PI * u2);
    if (cth_out) *cth_out = cth;
    if (sth_out) *sth_out = sth;
    if (cphi_out) *cphi_out = cphi;
    double mu_new = mu * cth + std::sqrt((1.0 - mu) * (1.0 + mu)) * sth * cphi;
    if (mu_new > 1.0) mu_new = 1.0;
    if (mu_new < -1.0) mu_new = -1.0;
    return mu_new;
}

// ---------------------------------------------------------------------------
// Next-event (peel-off) estimate of the detector tally.
//
// The detector of eq. 19 counts photons that leave the top inside the cone
// mu >= cos(alpha).  A photon leaving a scattering or reflection at depth T
// with direction cosine mu' > 0 escapes without further interaction with
// probability exp(-T/mu') (Beer-Lambert, eq. 7), so the expected detected
// weight of that event's outgoing flight is
//     w a E[ 1(mu' >= cos alpha) exp(-T/mu') ],
// a the albedo of the event, the expectation over the new direction (the
// phase function with a uniform azimuth, eq. 13-16, or the surface law).
// Summed over all events of all packets this has the expectation of the
// detector tally, because every detected photon left its last event that
// way.  Its apparent velocity is the path's value after the event, eq. 4.
//
// The expectation is estimated with one draw restricted to the directions
// that can reach the cone, each with its probability as weight:
//   surface, uniform polar angle: psi uniform on [0, alpha], weight
//     alpha / (pi/2);
//   surface, Lambert: u = mu'^2 uniform on [cos^2 alpha, 1], weight
//     sin^2 alpha;
//   particle: the cone lies within alpha of the vertical, so the scattering
//     angle Theta (measured from the incoming direction, at angle
//     Theta_0 = acos(mu) from the vertical) lies in
//     [max(0, Theta_0 - alpha), min(pi, Theta_0 + alpha)].  Theta is drawn
//     from the phase function restricted to that range (weight: its
//     probability M), then the azimuth from the arc where the new direction
//     is inside the cone: mu' = mu cos Theta + sqrt(1-mu^2) sin Theta cos phi
//     >= cos alpha  <=>  |phi| <= phi_c, phi_c = acos(kappa),
//     kappa = (cos alpha - mu cos Theta) / (sqrt(1-mu^2) sin Theta)
//     (weight phi_c / pi).
// Every weight lies in [0, 1], so the variance stays bounded.  The draw uses
// its own Philox block, counter word 0 = event index with the top bit set,
// so the analog or implicit transport is untouched.
// ---------------------------------------------------------------------------

// Henyey-Greenstein P(cos Theta <= x), written without cancellation:
// (1-g)(1+x) / (r (1 + g + r)), r = sqrt(1 + g^2 - 2 g x).  Equals the
// inverse of hg_angle's map from u to cos Theta.
double hg_cdf(double g, double x) {
    const double D = 1.0 + g * g - 2.0 * g * x;
    const double r = std::sqrt(D > 0.0 ? D : 0.0);
    const double den = r * (1.0 + g + r);
    return den > 0.0 ? (1.0 - g) * (1.0 + x) / den : 1.0;
}

// Table law: probability that the angle lies below theta (the CDF of the
// uniform-in-cell law, in units of 2^32).
double table_cdf32(const oracle_params& p, double theta) {
    const int n_cells = p.n_angles - 1;
    const double x = theta / (PI / (double)n_cells);
    if (x <= 0.0) return 0.0;
    if (x >= (double)n_cells) return 4294967296.0;
    int j = (int)std::floor(x);
    if (j > n_cells - 1) j = n_cells - 1;
    return (double)p.cdf[j] + (x - (double)j) * (double)(p.cdf[j + 1] - p.cdf[j]);
}

// Angle of the table law at CDF value y (units of 2^32): inside the cell
// holding y the angle is linear in y.
double table_theta_at(const oracle_params& p, double y) {
    int lo = 0, hi = p.n_angles - 2;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if ((double)p.cdf[mid] <= y) lo = mid; else hi = mid - 1;
    }
    const double width = (double)(p.cdf[lo + 1] - p.cdf[lo]);
    const double f = width > 0.0 ? (y - (double)p.cdf[lo]) / width : 0.0;
    return ((double)lo + f) * (PI / (double)(p.n_angles - 1));
}

// One restricted draw after a particle scattering of a photon with direction
// cosine mu at depth T; returns the weight (probability times attenuation)
// and the new cosine.
double peel_particle(const oracle_params& p, double mu, double T, double ur, double uphi, double* mu_out) {
    const double cos_a = p.cos_cone;
    const double alpha = std::acos(cos_a);
    const double theta0 = std::acos(mu);
    const double th_lo = std::fmax(0.0, theta0 - alpha), th_hi = std::fmin(PI, theta0 + alpha);
    double cth, sth, M;
    if (p.phase_kind == PHASE_TABLE) {
        const double y_lo = table_cdf32(p, th_lo), y_hi = table_cdf32(p, th_hi);
        M = (y_hi - y_lo) / 4294967296.0;
        const double th = table_theta_at(p, y_lo + (y_hi - y_lo) * ur);
        cth = std::cos(th);
        sth = std::sin(th);
    } else {
        const double g = p.hg_g;
        const double u_lo = hg_cdf(g, std::cos(th_hi)), u_hi = hg_cdf(g, std::cos(th_lo));
        M = u_hi - u_lo;
        hg_angle(g, u_lo + (u_hi - u_lo) * ur, &cth, &sth);
    }
    const double sm = std::sqrt(std::fmax(0.0, (1.0 - mu) * (1.0 + mu)));
    const double den = sm * sth;
    double phi_c;
    if (den <= 1e-300) {
        phi_c = PI;                       // every azimuth gives mu' = mu cos Theta
    } else {
        const double kappa = (cos_a - mu * cth) / den;
        phi_c = kappa <= -1.0 ? PI : (kappa >= 1.0 ? 0.0 : std::acos(kappa));
    }
    double mu_new = mu * cth + den * std::cos(phi_c * uphi);
    if (mu_new > 1.0) mu_new = 1.0;
    *mu_out = mu_new;
    if (!(M > 0.0) || phi_c <= 0.0 || mu_new <= 0.0) return 0.0;
    return M * (phi_c / PI) * std::exp(-T / mu_new);
}

// One restricted draw after a surface reflection (depth tau_total); returns
// the weight and the new cosine with its complement 1 - mu'.
double peel_surface(const oracle_params& p, double ur, double* mu_out, double* omc_out) {
    const double cos_a = p.cos_cone;
    double mu_new, omc, M;
    if (p.surface_law == SURFACE_LAMBERT) {
        const double s2 = (1.0 - cos_a) * (1.0 + cos_a);       // sin^2 alpha
        const double u = 1.0 - s2 * (1.0 - ur);
        mu_new = std::sqrt(u);
        omc = s2 * (1.0 - ur) / (1.0 + mu_new);
        M = s2;
    } else {
        const double alpha = std::acos(cos_a);
        const double psi = alpha * ur;
        const double sh = std::sin(0.5 * psi);
        mu_new = std::cos(psi);
        omc = 2.0 * sh * sh;
        M = alpha / (0.5 * PI);
    }
    *mu_out = mu_new;
    *omc_out = omc;
    if (mu_new <= 0.0) return 0.0;
    return M * std::exp(-p.tau_total / mu_new);
}

// Score a next-event estimate c at apparent velocity v (first_kind: 1 for a
// packet's first particle scattering with no surface hit before, 2 for its
// first surface hit with no scattering before, 0 otherwise).
void score_peel(const oracle_params& p, double c, double v, int first_kind, Tally& t) {
    const double dv = (p.v_hi - p.v_lo) / (double)p.n_bins;
    const double b = std::floor((v - p.v_lo) / dv);
    if (b < 0.0) {
        t.peel_sinks[0] += c;
    } else if (b >= (double)p.n_bins) {
        t.peel_sinks[1] += c;
    } else {
        const int ib = (int)b;
        t.P[ib] += c;
        t.P2[ib] += c * c;
        if (first_kind == 1 && !t.Ps.empty()) t.Ps[ib] += c;
        if (first_kind == 2 && !t.Psurf.empty()) t.Psurf[ib] += c;
    }
}

// The two uniforms of event k's next-event draw.
void peel_uniforms(const oracle_params& p, uint32_t k, uint32_t pid_lo, uint32_t pid_hi, double* ur, double* uphi) {
    const uint32_t key[2] = {(uint32_t)(p.seed & 0xffffffffu), (uint32_t)(p.seed >> 32)};
    const uint32_t ctr[4] = {k | 0x80000000u, pid_lo, pid_hi, p.stream};
    uint32_t X[4];
    philox4x32_10(ctr, key, X);
    *ur = uniform_from_word(X[0]);
    *uphi = uniform_from_word(X[1]);
}

void run_packet(const oracle_params& p, uint64_t pid, Tally& t) {
    const uint32_t key[2] = {(uint32_t)(p.seed & 0xffffffffu), (uint32_t)(p.seed >> 32)};
    const uint32_t pid_lo = (uint32_t)(pid & 0xffffffffu), pid_hi = (uint32_t)(pid >> 32);
    const uint32_t thr_albedo = (uint32_t)std::fmin(std::floor(p.albedo * 4294967296.0), 4294967295.0);
    const uint32_t thr_surface = (uint32_t)std::fmin(std::floor(p.surface_albedo * 4294967296.0), 4294967295.0);
    const bool albedo_one = p.albedo >= 1.0, surface_one = p.surface_albedo >= 1.0;

    double T = 0.0, mu = -1.0, w = 1.0;
    double big = 0.0, small = 0.0;   // apparent velocity = big - small
    int n_sc = 0, n_surf = 0;
    t.counts[CNT_PACKETS] += 1;
    Fp32Bound fb;                    // kept only for detected lists

    for (uint32_t k = 0;; ++k) {
        const uint32_t ctr[4] = {k, pid_lo, pid_hi, p.stream};
        uint32_t X[4];
        philox4x32_10(ctr, key, X);
        t.counts[CNT_FLIGHTS] += 1;
        const double u0 = uniform_from_word(X[0]);
        const double u1 = uniform_from_word(X[1]);
        const double u2 = uniform_from_word(X[2]);

        // Free flight: optical path s ~ Exp(1) (Beer-Lambert), vertical
        // depth change -s*mu.
        const double s = -std::log(u0);
        const double Tn = T - s * mu;

        if (mu < 0.0 && Tn >= p.tau_total) {
            // ---- free surface ----
            t.counts[CNT_SURFACE] += 1;
            double mu_new, one_minus_mu_new;
            if (p.surface_law == SURFACE_LAMBERT) {
                double r = std::sqrt(u1);
                mu_new = r;
                one_minus_mu_new = (1.0 - u1) / (1.0 + r);
            } else {
                double psi = 0.5 * PI * u1;
                double sh = std::sin(0.5 * psi);
                mu_new = std::cos(psi);
                one_minus_mu_new = 2.0 * sh * sh;
            }
            if (p.peel) {
                double ur, uphi, mp, omc_p;
                peel_uniforms(p, k, pid_lo, pid_hi, &ur, &uphi);
                const double c = w * p.surface_albedo * peel_surface(p, ur, &mp, &omc_p);
                const double v = (big + 0.5 * p.v_surface * (1.0 - mu)) - (small + 0.5 * p.v_surface * omc_p);
                score_peel(p, c, v, (n_sc == 0 && n_surf == 0) ? 2 : 0, t);
            }
            if (p.weighting == WEIGHT_ANALOG) {
                if (!surface_one && X[3] >= thr_surface) {
                    t.sinks[SINK_ABSORBED_SURFACE] += w;
                    return;
                }
            } else {
                t.sinks[SINK_ABSORBED_SURFACE] += w * (1.0 - p.surface_albedo);
                w *= p.surface_albedo;
            }
            if (t.keep_list) {
                const double U = Fp32Bound::U;
                const bool lambert = p.surface_law == SURFACE_LAMBERT;
                const double e_omc = (lambert ? 6.0 : 9.0) * U * one_minus_mu_new;
                const double e_mu = lambert ? 2.0 * U * mu_new : e_omc + U;
                fb.surface(p.v_surface, mu, one_minus_mu_new, e_omc, e_mu, p.tau_total,
                           big + 0.5 * p.v_surface * (1.0 - mu), small + 0.5 * p.v_surface * one_minus_mu_new);
            }
            big += 0.5 * p.v_surface * (1.0 - mu);
            small += 0.5 * p.v_surface * one_minus_mu_new;
            mu = mu_new;
            T = p.tau_total;
            n_surf += 1;
            continue;
        }
        if (mu > 0.0 && Tn <= 0.0) {
            // ---- leaves the top of the cloud ----
            t.counts[CNT_EXITS] += 1;
            if (mu >= p.cos_cone) {
                t.counts[CNT_DETECTED] += 1;
                const double v = big - small;
                const double dv = (p.v_hi - p.v_lo) / (double)p.n_bins;
                const double b = std::floor((v - p.v_lo) / dv);
                if (b < 0.0) {
                    t.sinks[SINK_UNDER] += w;
                } else if (b >= (double)p.n_bins) {
                    t.sinks[SINK_OVER] += w;
                } else {
                    const int ib = (int)b;
                    t.W[ib] += w;
                    t.W2[ib] += w * w;
                    if (!t.Ws.empty() && n_sc == 1 && n_surf == 0) t.Ws[ib] += w;
                    if (!t.Wsurf.empty() && n_sc == 0 && n_surf == 1) t.Wsurf[ib] += w;
                }
                if (t.keep_list) {
                    // beat phase from the reserved last event block of this packet
                    const uint32_t pctr[4] = {0xffffffffu, pid_lo, pid_hi, p.stream};
                    uint32_t P[4];
                    philox4x32_10(pctr, key, P);
                    t.lw.push_back(w);
                    t.lv.push_back(v);
                    t.lph.push_back((double)P[0] * (1.0 / 4294967296.0));
                    t.lpid.push_back(pid);
                    t.lerr.push_back(fb.eBig + fb.eSmall);
                }
            } else {
                t.sinks[SINK_UNDETECTED] += w;
            }
            return;
        }

        // ---- interaction with a particle at depth Tn ----
        t.counts[CNT_COLLISIONS] += 1;
        const double V = zeta_at_depth(p, Tn);
        if (n_sc == p.max_orders) {
            t.sinks[SINK_TRUNCATED] += w;
            return;
        }
        if (p.peel) {
            double ur, uphi, mp;
            peel_uniforms(p, k, pid_lo, pid_hi, &ur, &uphi);
            const double c = w * p.albedo * peel_particle(p, mu, Tn, ur, uphi, &mp);
            const double v = (big + 0.5 * V * (1.0 - mu)) - (small + 0.5 * V * (1.0 - mp));
            score_peel(p, c, v, (n_sc == 0 && n_surf == 0) ? 1 : 0, t);
        }
        if (p.weighting == WEIGHT_ANALOG) {
            if (!albedo_one && X[3] >= thr_albedo) {
                t.sinks[SINK_ABSORBED_PARTICLE] += w;
                return;
            }
        } else {
            t.sinks[SINK_ABSORBED_PARTICLE] += w * (1.0 - p.albedo);
            w *= p.albedo;
        }
        n_sc += 1;

        double cth = 0.0, sth = 0.0, cphi = 0.0;
        const double mu_new = scattered_mu(p, mu, X[1], u1, u2, &cth, &sth, &cphi);
        if (t.keep_list) {
            // FP32 errors of the polar angle's cosine and sine: a tabulated
            // angle comes from the hardware cosine and sine of the cell
            // position; the HG cosine from its inversion (expanded form
            // below |g| = 0.1, direct form above, whose rounding is divided
            // by 2|g|), its sine as sqrt((1 - x)(1 + x))
            const double U = Fp32Bound::U;
            double ex, es;
            if (p.phase_kind == PHASE_TABLE) {
                ex = es = 4.0 * U * std::acos(cth) + 4.0 * U;
            } else {
                const double g = p.hg_g;
                if (std::fabs(g) < 0.1) {
                    ex = 8.0 * U;
                } else {
                    const double q = (1.0 - g * g) / (1.0 - g + 2.0 * g * u1);
                    ex = (6.0 * U * q * q + U * (1.0 + g * g) + U * std::fabs(1.0 + g * g - q * q)) /
                         (2.0 * std::fabs(g)) + 2.0 * U;
                }
                es = Fp32Bound::sine_err(cth, sth, ex);
            }
            const int j = find_layer(p, Tn);
            const double slope = (p.v_top - p.v_bottom) / p.n_layers / (p.T[j + 1] - p.T[j]);
            fb.collision(fb.flight(-std::log(u0), mu, Tn), Tn, slope, V, mu, cth, sth, ex, es, cphi, mu_new,
                         big + 0.5 * V * (1.0 - mu), small + 0.5 * V * (1.0 - mu_new));
        }
        big += 0.5 * V * (1.0 - mu);
        small += 0.5 * V * (1.0 - mu_new);
        mu = mu_new;
        T = Tn;
    }
}

void run_range(const oracle_params* p, uint64_t begin, uint64_t end, Tally* t) {
    for (uint64_t pid = begin; pid < end; ++pid) run_packet(*p, pid, *t);
}

}  // namespace

extern "C" {

// Returns 0 on success, -1 on invalid arguments.
int oracle_run(const oracle_params* p, oracle_out* out) {
    if (!p || !out || p->n_bins < 1 || p->n_layers < 1 || !p->T || !out->W || !out->W2) return -1;
    if (p->phase_kind == PHASE_TABLE && (!p->cdf || p->n_angles < 2)) return -1;
    if (p->peel && (!out->P || !out->P2)) return -1;
    int nt = p->n_threads > 0 ? p->n_threads : 1;
    if ((uint64_t)nt > p->n_packets && p->n_packets > 0) nt = (int)p->n_packets;
    if (nt < 1) nt = 1;
    std::vector<Tally> tallies(nt);
    for (auto& t : tallies) {
        t.W.assign(p->n_bins, 0.0);
        t.W2.assign(p->n_bins, 0.0);
        if (out->W_single) t.Ws.assign(p->n_bins, 0.0);
        if (out->W_surface) t.Wsurf.assign(p->n_bins, 0.0);
        t.keep_list = out->list_capacity > 0;
        if (p->peel) {
            t.P.assign(p->n_bins, 0.0);
            t.P2.assign(p->n_bins, 0.0);
            if (out->P_single) t.Ps.assign(p->n_bins, 0.0);
            if (out->P_surface) t.Psurf.assign(p->n_bins, 0.0);
        }
    }
    std::vector<std::thread> threads;
    for (int i = 0; i < nt; ++i) {
        uint64_t b = p->pid_begin + p->n_packets * (uint64_t)i / (uint64_t)nt;
        uint64_t e = p->pid_begin + p->n_packets * (uint64_t)(i + 1) / (uint64_t)nt;
        threads.emplace_back(run_range, p, b, e, &tallies[i]);
    }
    for (auto& th : threads) th.join();

    for (int b = 0; b < p->n_bins; ++b) {
        out->W[b] = 0.0; out->W2[b] = 0.0;
        if (out->W_single) out->W_single[b] = 0.0;
        if (out->W_surface) out->W_surface[b] = 0.0;
    }
    for (int s = 0; s < N_SINKS; ++s) out->sinks[s] = 0.0;
    for (int c = 0; c < N_COUNTS; ++c) out->counts[c] = 0;
    if (p->peel) {
        for (int b = 0; b < p->n_bins; ++b) {
            out->P[b] = 0.0;
            out->P2[b] = 0.0;
            if (out->P_single) out->P_single[b] = 0.0;
            if (out->P_surface) out->P_surface[b] = 0.0;
        }
        out->peel_sinks[0] = out->peel_sinks[1] = 0.0;
    }
    uint64_t n_list = 0;
    for (int i = 0; i < nt; ++i) {
        const Tally& t = tallies[i];
        for (int b = 0; b < p->n_bins; ++b) {
            out->W[b] += t.W[b];
            out->W2[b] += t.W2[b];
            if (out->W_single) out->W_single[b] += t.Ws[b];
            if (out->W_surface) out->W_surface[b] += t.Wsurf[b];
        }
        if (p->peel) {
            for (int b = 0; b < p->n_bins; ++b) {
                out->P[b] += t.P[b];
                out->P2[b] += t.P2[b];
                if (out->P_single) out->P_single[b] += t.Ps[b];
                if (out->P_surface) out->P_surface[b] += t.Psurf[b];
            }
            out->peel_sinks[0] += t.peel_sinks[0];
            out->peel_sinks[1] += t.peel_sinks[1];
        }
        for (int s = 0; s < N_SINKS; ++s) out->sinks[s] += t.sinks[s];
        for (int c = 0; c < N_COUNTS; ++c) out->counts[c] += t.counts[c];
        for (size_t j = 0; j < t.lw.size(); ++j, ++n_list) {
            if (n_list < out->list_capacity) {
                if (out->list_w) out->list_w[n_list] = t.lw[j];
                if (out->list_v) out->list_v[n_list] = t.lv[j];
                if (out->list_phase) out->list_phase[n_list] = t.lph[j];
                if (out->list_pid) out->list_pid[n_list] = t.lpid[j];
                if (out->list_err32) out->list_err32[n_list] = t.lerr[j];
            }
        }
    }
    out->list_count = n_list;
    return 0;
}

}  // extern "C"

extern "C" {

// Test hook: the scattering-angle sampler alone.  Draw i uses the Philox
// block with counter (i, 0, 0, stream) and the same words the transport uses
// (X[1] for the table cell, u1 for Henyey-Greenstein).
int oracle_sample_scatter(const oracle_params* p, uint64_t n, double* cos_out) {
    if (!p || !cos_out) return -1;
    if (p->phase_kind == PHASE_TABLE && (!p->cdf || p->n_angles < 2)) return -1;
    const uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), 0u, p->stream};
        uint32_t X[4];
        philox4x32_10(ctr, key, X);
        double c, sn;
        if (p->phase_kind == PHASE_TABLE) table_angle(*p, X[1], &c, &sn);
        else hg_angle(p->hg_g, uniform_from_word(X[1]), &c, &sn);
        cos_out[i] = c;
    }
    return 0;
}

}  // extern "C"

extern "C" {

// Test hook: one scattering of a packet travelling with direction cosine
// mu_in; draw i uses the Philox block with counter (i, 1, 0, stream).
int oracle_scatter_direction(const oracle_params* p, double mu_in, uint64_t n, double* mu_out) {
    if (!p || !mu_out || mu_in < -1.0 || mu_in > 1.0) return -1;
    if (p->phase_kind == PHASE_TABLE && (!p->cdf || p->n_angles < 2)) return -1;
    const uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t ctr[4] = {(uint32_t)i, 1u, (uint32_t)(i >> 32), p->stream};
        uint32_t X[4];
        philox4x32_10(ctr, key, X);
        mu_out[i] = scattered_mu(*p, mu_in, X[1], uniform_from_word(X[1]), uniform_from_word(X[2]));
    }
    return 0;
}

}  // extern "C"

extern "C" {

// Test hook: n next-event draws after a particle scattering (surface != 0:
// a surface reflection) of a photon with direction cosine mu_in at depth T;
// draw i uses the Philox block with counter (i, 2, 0, stream).  w_out[i]
// receives the draw's weight (probability times attenuation, before the
// albedo), mu_out[i] its new cosine.
int oracle_peel_draws(const oracle_params* p, int surface, double mu_in, double T, uint64_t n, double* w_out,
                      double* mu_out) {
    if (!p || !w_out || !mu_out || mu_in < -1.0 || mu_in > 1.0) return -1;
    if (p->phase_kind == PHASE_TABLE && (!p->cdf || p->n_angles < 2)) return -1;
    const uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t ctr[4] = {(uint32_t)i, 2u, (uint32_t)(i >> 32), p->stream};
        uint32_t X[4];
        philox4x32_10(ctr, key, X);
        const double ur = uniform_from_word(X[0]), uphi = uniform_from_word(X[1]);
        if (surface) {
            double omc;
            w_out[i] = peel_surface(*p, ur, &mu_out[i], &omc);
        } else {
            w_out[i] = peel_particle(*p, mu_in, T, ur, uphi, &mu_out[i]);
        }
    }
    return 0;
}

}  // extern "C"

// ===========================================================================
// The paper's own procedure as a fidelity mode (Sec. II.B, steps 2-7).
//
// Where the estimator above samples each free flight exactly, the paper moves
// every photon by a fixed step of one thousandth of the cloud height (one
// layer thickness) along its direction and lets it cross that step with the
// Beer-Lambert probability of eq. 10 (one random number per step); a photon
// that does not cross interacts at the end of its step (eq. 11).  The polar
// angle comes from acceptance-rejection against the phase function (step 4).
// The surface, Doppler, weighting and detector rules are those above.
//
// This mode draws a variable number of random numbers, so it uses its own
// stream (consecutive words of the packet's Philox blocks, counter word 3 =
// stream with its top bit flipped) and agrees with the exact estimator in
// distribution only: tests compare the two statistically.  Reading of the
// step: its length is (v_top - v_bottom) / n_layers in the velocity
// coordinate, cut at the slab's faces; a photon running parallel to the
// layers sees the extinction of its layer along the whole step.
// ===========================================================================
namespace {

struct WordStream {
    uint32_t key[2];
    uint32_t pid_lo, pid_hi, stream;
    uint32_t k = 0, pos = 4;
    uint32_t buf[4];
    uint32_t next() {
        if (pos == 4) {
            const uint32_t ctr[4] = {k++, pid_lo, pid_hi, stream};
            philox4x32_10(ctr, key, buf);
            pos = 0;
        }
        return buf[pos++];
    }
    double uniform() { return uniform_from_word(next()); }
};

// Cumulative extinction depth from the top at velocity coordinate zeta
// (linear inside each layer).
double depth_at_zeta(const oracle_params& p, double zeta) {
    const double dz = (p.v_top - p.v_bottom) / p.n_layers;
    const double x = (p.v_top - zeta) / dz;
    if (x <= 0.0) return 0.0;
    if (x >= (double)p.n_layers) return p.T[p.n_layers];
    int j = (int)std::floor(x);
    if (j > p.n_layers - 1) j = p.n_layers - 1;
    return p.T[j] + (x - (double)j) * (p.T[j + 1] - p.T[j]);
}

// Extinction per unit of the velocity coordinate in the layer holding zeta.
double extinction_at_zeta(const oracle_params& p, double zeta) {
    const double dz = (p.v_top - p.v_bottom) / p.n_layers;
    int j = (int)std::floor((p.v_top - zeta) / dz);
    if (j < 0) j = 0;
    if (j > p.n_layers - 1) j = p.n_layers - 1;
    return (p.T[j + 1] - p.T[j]) / dz;
}

// Acceptance-rejection sampler of the polar angle.  Table: the density in
// theta is constant inside each cell and proportional to the cell's mass, so
// theta is proposed uniform on [0, pi] and kept with probability
// mass(cell) / max mass.  Henyey-Greenstein: cos(theta) is proposed uniform
// on [-1, 1] and kept with probability p(cos) / p_max, p_max = p(sign g).
struct ArSampler {
    std::vector<double> mass;
    double mass_max = 0.0;
    explicit ArSampler(const oracle_params& p) {
        if (p.phase_kind == PHASE_TABLE) {
            mass.resize(p.n_angles - 1);
            for (int j = 0; j + 1 < p.n_angles; ++j) {
                mass[j] = (double)(p.cdf[j + 1] - p.cdf[j]);
                if (mass[j] > mass_max) mass_max = mass[j];
            }
        }
    }
    void sample(const oracle_params& p, WordStream& rs, double* c, double* s) const {
        if (p.phase_kind == PHASE_TABLE) {
            const int n_cells = p.n_angles - 1;
            for (;;) {
                const double x = rs.uniform() * (double)n_cells;
                int j = (int)x;
                if (j > n_cells - 1) j = n_cells - 1;
                if (rs.uniform() * mass_max < mass[j]) {
                    const double theta = x * (PI / (double)n_cells);
                    *c = std::cos(theta);
                    *s = std::sin(theta);
                    return;
                }
            }
        }
        const double g = p.hg_g;
        const double pmax = g == 0.0 ? 1.0 : 1.0 / ((1.0 - std::fabs(g)) * (1.0 - std::fabs(g)) * (1.0 - std::fabs(g)));
        for (;;) {
            const double ct = 2.0 * rs.uniform() - 1.0;
            const double base = 1.0 + g * g - 2.0 * g * ct;
            const double dens = g == 0.0 ? 1.0 : 1.0 / (base * std::sqrt(base));
            if (rs.uniform() * pmax < dens) {
                *c = ct;
                const double s2 = (1.0 - ct) * (1.0 + ct);
                *s = std::sqrt(s2 > 0.0 ? s2 : 0.0);
                return;
            }
        }
    }
};

void tally_exit(const oracle_params& p, double w, double v, int n_sc, int n_surf, double mu, Tally& t) {
    t.counts[CNT_EXITS] += 1;
    if (mu < p.cos_cone) {
        t.sinks[SINK_UNDETECTED] += w;
        return;
    }
    t.counts[CNT_DETECTED] += 1;
    const double dv = (p.v_hi - p.v_lo) / (double)p.n_bins;
    const double b = std::floor((v - p.v_lo) / dv);
    if (b < 0.0) {
        t.sinks[SINK_UNDER] += w;
    } else if (b >= (double)p.n_bins) {
        t.sinks[SINK_OVER] += w;
    } else {
        const int ib = (int)b;
        t.W[ib] += w;
        t.W2[ib] += w * w;
        if (!t.Ws.empty() && n_sc == 1 && n_surf == 0) t.Ws[ib] += w;
        if (!t.Wsurf.empty() && n_sc == 0 && n_surf == 1) t.Wsurf[ib] += w;
    }
}

void run_packet_literal(const oracle_params& p, const ArSampler& ar, uint64_t pid, Tally& t) {
    WordStream rs;
    rs.key[0] = (uint32_t)(p.seed & 0xffffffffu);
    rs.key[1] = (uint32_t)(p.seed >> 32);
    rs.pid_lo = (uint32_t)(pid & 0xffffffffu);
    rs.pid_hi = (uint32_t)(pid >> 32);
    rs.stream = p.stream ^ 0x80000000u;
    const double step = (p.v_top - p.v_bottom) / p.n_layers;

    double zeta = p.v_top, mu = -1.0, w = 1.0, big = 0.0, small = 0.0;
    int n_sc = 0, n_surf = 0;
    t.counts[CNT_PACKETS] += 1;
    for (;;) {
        t.counts[CNT_FLIGHTS] += 1;
        // one step along the direction, cut at the faces of the slab
        double zeta_end = zeta + step * mu;
        int face = 0;
        if (zeta_end <= p.v_bottom) { zeta_end = p.v_bottom; face = -1; }
        else if (zeta_end >= p.v_top) { zeta_end = p.v_top; face = 1; }
        const double tau_step = std::fabs(mu) > 1e-12
            ? std::fabs(depth_at_zeta(p, zeta_end) - depth_at_zeta(p, zeta)) / std::fabs(mu)
            : step * extinction_at_zeta(p, zeta);
        const bool crosses = rs.uniform() < std::exp(-tau_step);
        zeta = zeta_end;
        if (crosses) {
            if (face == 1) {
                tally_exit(p, w, big - small, n_sc, n_surf, mu, t);
                return;
            }
            if (face == -1) {
                // diffuse reflection at the moving free surface
                t.counts[CNT_SURFACE] += 1;
                const double u1 = rs.uniform();
                double mu_new, one_minus_mu_new;
                if (p.surface_law == SURFACE_LAMBERT) {
                    const double r = std::sqrt(u1);
                    mu_new = r;
                    one_minus_mu_new = (1.0 - u1) / (1.0 + r);
                } else {
                    const double psi = 0.5 * PI * u1;
                    const double sh = std::sin(0.5 * psi);
                    mu_new = std::cos(psi);
                    one_minus_mu_new = 2.0 * sh * sh;
                }
                if (p.weighting == WEIGHT_ANALOG) {
                    if (rs.uniform() >= p.surface_albedo) {
                        t.sinks[SINK_ABSORBED_SURFACE] += w;
                        return;
                    }
                } else {
                    t.sinks[SINK_ABSORBED_SURFACE] += w * (1.0 - p.surface_albedo);
                    w *= p.surface_albedo;
                }
                big += 0.5 * p.v_surface * (1.0 - mu);
                small += 0.5 * p.v_surface * one_minus_mu_new;
                mu = mu_new;
                n_surf += 1;
            }
            continue;
        }
        // interaction at the end of the step
        t.counts[CNT_COLLISIONS] += 1;
        if (n_sc == p.max_orders) {
            t.sinks[SINK_TRUNCATED] += w;
            return;
        }
        if (p.weighting == WEIGHT_ANALOG) {
            if (rs.uniform() >= p.albedo) {
                t.sinks[SINK_ABSORBED_PARTICLE] += w;
                return;
            }
        } else {
            t.sinks[SINK_ABSORBED_PARTICLE] += w * (1.0 - p.albedo);
            w *= p.albedo;
        }
        n_sc += 1;
        double cth, sth;
        ar.sample(p, rs, &cth, &sth);
        const double cphi = std::cos(2.0 * PI * rs.uniform());
        double mu_new = mu * cth + std::sqrt((1.0 - mu) * (1.0 + mu)) * sth * cphi;
        if (mu_new > 1.0) mu_new = 1.0;
        if (mu_new < -1.0) mu_new = -1.0;
        const double V = zeta;
        big += 0.5 * V * (1.0 - mu);
        small += 0.5 * V * (1.0 - mu_new);
        mu = mu_new;
    }
}

void run_range_literal(const oracle_params* p, const ArSampler* ar, uint64_t begin, uint64_t end, Tally* t) {
    for (uint64_t pid = begin; pid < end; ++pid) run_packet_literal(*p, *ar, pid, *t);
}

}  // namespace

extern "C" {

// The literal procedure over the requested packets; the same outputs as
// oracle_run (no detected list; counts[flights] holds the steps taken).
int oracle_run_literal(const oracle_params* p, oracle_out* out) {
    if (!p || !out || p->n_bins < 1 || p->n_layers < 1 || !p->T || !out->W || !out->W2) return -1;
    if (p->phase_kind == PHASE_TABLE && (!p->cdf || p->n_angles < 2)) return -1;
    if (p->phase_kind == PHASE_HG && !(std::fabs(p->hg_g) < 1.0)) return -1;
    if (!(p->v_top > p->v_bottom)) return -1;
    const ArSampler ar(*p);
    int nt = p->n_threads > 0 ? p->n_threads : 1;
    if ((uint64_t)nt > p->n_packets && p->n_packets > 0) nt = (int)p->n_packets;
    if (nt < 1) nt = 1;
    std::vector<Tally> tallies(nt);
    for (auto& t : tallies) {
        t.W.assign(p->n_bins, 0.0);
        t.W2.assign(p->n_bins, 0.0);
        if (out->W_single) t.Ws.assign(p->n_bins, 0.0);
        if (out->W_surface) t.Wsurf.assign(p->n_bins, 0.0);
    }
    std::vector<std::thread> threads;
    for (int i = 0; i < nt; ++i) {
        uint64_t b = p->pid_begin + p->n_packets * (uint64_t)i / (uint64_t)nt;
        uint64_t e = p->pid_begin + p->n_packets * (uint64_t)(i + 1) / (uint64_t)nt;
        threads.emplace_back(run_range_literal, p, &ar, b, e, &tallies[i]);
    }
    for (auto& th : threads) th.join();
    for (int b = 0; b < p->n_bins; ++b) {
        out->W[b] = 0.0; out->W2[b] = 0.0;
        if (out->W_single) out->W_single[b] = 0.0;
        if (out->W_surface) out->W_surface[b] = 0.0;
    }
    for (int s = 0; s < N_SINKS; ++s) out->sinks[s] = 0.0;
    for (int c = 0; c < N_COUNTS; ++c) out->counts[c] = 0;
    for (int i = 0; i < nt; ++i) {
        const Tally& t = tallies[i];
        for (int b = 0; b < p->n_bins; ++b) {
            out->W[b] += t.W[b];
            out->W2[b] += t.W2[b];
            if (out->W_single) out->W_single[b] += t.Ws[b];
            if (out->W_surface) out->W_surface[b] += t.Wsurf[b];
        }
        for (int s = 0; s < N_SINKS; ++s) out->sinks[s] += t.sinks[s];
        for (int c = 0; c < N_COUNTS; ++c) out->counts[c] += t.counts[c];
    }
    out->list_count = 0;
    return 0;
}

// Test hook: cos(Theta) from the acceptance-rejection sampler alone, n draws
// from one word stream (packet id 0).
int oracle_sample_scatter_ar(const oracle_params* p, uint64_t n, double* cos_out) {
    if (!p || !cos_out) return -1;
    if (p->phase_kind == PHASE_TABLE && (!p->cdf || p->n_angles < 2)) return -1;
    if (p->phase_kind == PHASE_HG && !(std::fabs(p->hg_g) < 1.0)) return -1;
    const ArSampler ar(*p);
    WordStream rs;
    rs.key[0] = (uint32_t)(p->seed & 0xffffffffu);
    rs.key[1] = (uint32_t)(p->seed >> 32);
    rs.pid_lo = 0;
    rs.pid_hi = 0;
    rs.stream = p->stream ^ 0x80000000u;
    for (uint64_t i = 0; i < n; ++i) {
        double c, s;
        ar.sample(*p, rs, &c, &s);
        cos_out[i] = c;
    }
    return 0;
}

}  // extern "C"
