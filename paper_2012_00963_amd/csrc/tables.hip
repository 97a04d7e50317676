// Set tables on the device (FP64): layer depths, Mie optics, phase CDF.
//
//  * Layer depths (Sec. II.B step 2 and eq. 8): the slab in zeta = z/t is cut
//    into n equal layers; each layer's extinction depth is tau_total times
//    the exact integral of the density over the layer divided by the column
//    total (uniform, exponential eq. 20, or caller weights).  T[j] is the
//    depth from the top at the upper edge of layer j.  A guide over uniform
//    depth cells (guide[i] = last layer with T[j] <= i tau/G) bounds the
//    search of the transport kernel.
//  * Mie optics (eq. 12-14): Gauss-Legendre nodes over ln d (eq. 21 sizes);
//    per size parameter x = pi d / lambda the coefficients a_n, b_n from
//    Riccati-Bessel functions with the logarithmic derivative D_n(mx) taken
//    by downward recurrence (Bohren & Huffman ch. 4; series length
//    x + 4 x^(1/3) + 2 after Wiscombe 1980), efficiencies Q_ext, Q_sca, the
//    asymmetry g, and the intensity |S1|^2 + |S2|^2 at every tabulated angle
//    (pi_n, tau_n by upward recurrence).  The size-resolved intensities form
//    a basis kept on the device; a set's phase function is its weight
//    vector times the basis, its albedo <C_sca>/<C_ext> (eq. 11).
//  * Phase CDF: cell masses are trapezoids of p(theta) sin(theta) on
//    theta_j = j pi/(n-1); the CDF is rounded to integers C_j = round(2^32
//    F_j) so the transport kernel picks cells by integer comparison; a guide
//    over the top bits of the 32-bit draw bounds the search.
#include "pdv_device.h"
#include "pdv_internal.h"

namespace pdv {

constexpr double PI_D = 3.14159265358979323846;

struct Cplx {
    double re, im;
};
__device__ __forceinline__ Cplx cmk(double r, double i) { return Cplx{r, i}; }
__device__ __forceinline__ Cplx operator+(Cplx a, Cplx b) { return cmk(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ Cplx operator-(Cplx a, Cplx b) { return cmk(a.re - b.re, a.im - b.im); }
__device__ __forceinline__ Cplx operator*(Cplx a, Cplx b) {
    return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__device__ __forceinline__ Cplx operator*(double s, Cplx a) { return cmk(s * a.re, s * a.im); }
__device__ __forceinline__ Cplx cdiv(Cplx a, Cplx b) {
    // Smith's algorithm
    if (fabs(b.re) >= fabs(b.im)) {
        const double r = b.im / b.re, den = b.re + b.im * r;
        return cmk((a.re + a.im * r) / den, (a.im - a.re * r) / den);
    } else {
        const double r = b.re / b.im, den = b.re * r + b.im;
        return cmk((a.re * r + a.im) / den, (a.im * r - a.re) / den);
    }
}
__device__ __forceinline__ double cabs2(Cplx a) { return a.re * a.re + a.im * a.im; }

// --------------------------------------------------------------------------
// Layer table: one block per set.
// --------------------------------------------------------------------------

// Depth of guide point i, and the first guide point at or below depth T
// (the smallest i in [0, G+1] with tau i / G >= T), found from an estimate
// and corrected with the same expression.
__device__ __forceinline__ double guide_depth(double tau, int i) {
    return tau * (double)i / (double)LAYER_GUIDE;
}
__device__ int first_cell_at_or_above(double tau, double T) {
    if (!(tau > 0.0)) return T <= 0.0 ? 0 : LAYER_GUIDE + 1;
    double e = ceil(T / tau * (double)LAYER_GUIDE);
    int i = e < 0.0 ? 0 : (e > (double)(LAYER_GUIDE + 1) ? LAYER_GUIDE + 1 : (int)e);
    while (i > 0 && guide_depth(tau, i - 1) >= T) --i;
    while (i <= LAYER_GUIDE && guide_depth(tau, i) < T) ++i;
    return i;
}

__global__ void __launch_bounds__(1024)
layer_table_kernel(const LayerJob* __restrict__ jobs, const double* __restrict__ density, uint8_t* tables) {
    const LayerJob J = jobs[blockIdx.x];
    const int n = J.n_layers;
    uint8_t* tb = tables + J.tab_offset;
    float* T32 = (float*)(tb + TableLayout::T32);
    double* T64 = (double*)(tb + TableLayout::T64);
    uint16_t* lg = (uint16_t*)(tb + TableLayout::LGUIDE);
    __shared__ double s_mass[MAX_LAYERS];
    __shared__ double s_part[1024];
    const int tid = threadIdx.x, nt = blockDim.x;

    for (int j = tid; j < n; j += nt) {
        double m;
        if (J.density_kind == 1) {
            // exact integral of exp(-(zeta - v_bottom)/v0) over the layer
            const double span = J.v_top - J.v_bottom;
            const double z_hi = J.v_top - span * (double)j / (double)n;
            const double z_lo = J.v_top - span * (double)(j + 1) / (double)n;
            m = J.v0 * (exp(-(z_lo - J.v_bottom) / J.v0) - exp(-(z_hi - J.v_bottom) / J.v0));
        } else if (J.density_kind == 2) {
            m = density[J.density_offset + (uint64_t)(n - 1 - j)];   // bottom-up input
        } else {
            m = 1.0;
        }
        s_mass[j] = m;
    }
    __syncthreads();
    // inclusive scan: each thread sums a contiguous chunk, then the chunk sums
    const int per = (n + nt - 1) / nt;
    const int b0 = tid * per, b1 = min(n, b0 + per);
    double local = 0.0;
    for (int j = b0; j < b1; ++j) local += s_mass[j];
    s_part[tid] = local;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        const double v = tid >= off ? s_part[tid - off] : 0.0;
        __syncthreads();
        s_part[tid] += v;
        __syncthreads();
    }
    const double total = s_part[nt - 1];
    double run = tid > 0 ? s_part[tid - 1] : 0.0;
    for (int j = b0; j < b1; ++j) {
        run += s_mass[j];
        const double t = (j + 1 == n) ? J.tau_total : run / total * J.tau_total;
        T64[j + 1] = t;
        T32[j + 1] = (float)t;
        s_mass[j] = t;            // s_mass[j] now holds T[j+1]
    }
    if (tid == 0) { T64[0] = 0.0; T32[0] = 0.0f; }
    __syncthreads();
    // guide over uniform depth cells: lg[i] = last layer j with T[j] <= t_i,
    // t_i = tau i / G; every layer writes the entries whose t_i falls inside it
    for (int j = tid; j < n; j += nt) {
        const int lo = first_cell_at_or_above(J.tau_total, j == 0 ? 0.0 : s_mass[j - 1]);
        const int hi = j + 1 < n ? first_cell_at_or_above(J.tau_total, s_mass[j]) : LAYER_GUIDE + 1;
        for (int i = lo; i < hi; ++i) lg[i] = (uint16_t)j;
    }
}

// --------------------------------------------------------------------------
// Gauss-Legendre nodes on [-1, 1] by Newton iteration on P_n.
// --------------------------------------------------------------------------
__global__ void gauss_legendre_kernel(int n, double* __restrict__ x_out, double* __restrict__ w_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // i-th root from the top, initial guess cos(pi (i + 0.75)/(n + 0.5))
    double x = cos(PI_D * ((double)i + 0.75) / ((double)n + 0.5));
    double dp = 1.0;
    for (int iter = 0; iter < 12; ++iter) {
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / (double)k;
            p0 = p1; p1 = p2;
        }
        const double pn = n == 1 ? x : p1, pn1 = n == 1 ? 1.0 : p0;
        dp = (double)n * (x * pn - pn1) / (x * x - 1.0);
        const double dx = pn / dp;
        x -= dx;
        if (fabs(dx) <= 4e-16) break;
    }
    // recompute the derivative at the converged root
    {
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / (double)k;
            p0 = p1; p1 = p2;
        }
        const double pn = n == 1 ? x : p1, pn1 = n == 1 ? 1.0 : p0;
        dp = (double)n * (x * pn - pn1) / (x * x - 1.0);
    }
    // ascending order like the usual convention
    const int o = n - 1 - i;
    x_out[o] = x;
    w_out[o] = 2.0 / ((1.0 - x * x) * dp * dp);
}

// --------------------------------------------------------------------------
// Mie basis: sizes on Gauss-Legendre nodes in ln d over [d_min, d_max].
// Layout: coef[n][i] (n = 1..nmax at index n-1), basis[i][j] (node-major).
// --------------------------------------------------------------------------

__global__ void mie_nodes_kernel(int n, const double* __restrict__ gl_x, const double* __restrict__ gl_w,
                                 double ln_dmin, double ln_dmax, double wavelength, MieNodeInfo* info) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double half = 0.5 * (ln_dmax - ln_dmin), mid = 0.5 * (ln_dmax + ln_dmin);
    const double lnd = half * gl_x[i] + mid;
    MieNodeInfo I;
    I.lnd = lnd;
    I.wq = half * gl_w[i];
    I.x = PI_D * exp(lnd) / wavelength;
    I.nstop = (int)floor(I.x + 4.0 * cbrt(I.x) + 2.0);
    I.q_ext = I.q_sca = I.g = 0.0;
    I.pad = 0;
    info[i] = I;
}

// One thread per size: D_n(mx) downward (stored temporarily in the a slots),
// then psi_n, xi_n upward and a_n, b_n; efficiencies and asymmetry.
__global__ void mie_coef_kernel(int n_nodes, int nmax, int nmx_max, double m_re, double m_im,
                                MieNodeInfo* __restrict__ info, Cplx* __restrict__ coef_a, Cplx* __restrict__ coef_b,
                                Cplx* __restrict__ dscratch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nodes) return;
    MieNodeInfo I = info[i];
    const double x = I.x;
    const Cplx m = cmk(m_re, m_im);
    const Cplx mx = cmk(m_re * x, m_im * x);
    const int nstop = I.nstop;
    const double amx = sqrt(mx.re * mx.re + mx.im * mx.im);
    int nmx = (int)fmax((double)nstop, ceil(amx)) + 16;
    if (nmx > nmx_max) nmx = nmx_max;
    // downward recurrence D_{n-1} = n/mx - 1/(D_n + n/mx), D_nmx = 0
    Cplx D = cmk(0.0, 0.0);
    for (int k = nmx; k >= 1; --k) {
        const Cplx n_over = cdiv(cmk((double)k, 0.0), mx);
        if (k <= nstop) dscratch[(uint64_t)(k - 1) * n_nodes + i] = D;   // D_k
        D = n_over - cdiv(cmk(1.0, 0.0), D + n_over);
    }
    double psi_m1 = cos(x), psi_0 = sin(x);
    double chi_m1 = -sin(x), chi_0 = cos(x);
    double s_ext = 0.0, s_sca = 0.0, s_g = 0.0;
    Cplx a_prev = cmk(0.0, 0.0), b_prev = cmk(0.0, 0.0);
    for (int k = 1; k <= nmax; ++k) {
        Cplx an = cmk(0.0, 0.0), bn = cmk(0.0, 0.0);
        if (k <= nstop) {
            const double psi_n = (2.0 * k - 1.0) / x * psi_0 - psi_m1;
            const double chi_n = (2.0 * k - 1.0) / x * chi_0 - chi_m1;
            const Cplx xi_n = cmk(psi_n, -chi_n);
            const Cplx xi_p = cmk(psi_0, -chi_0);
            const Cplx Dk = dscratch[(uint64_t)(k - 1) * n_nodes + i];
            const Cplx n_x = cmk((double)k / x, 0.0);
            const Cplx ta = cdiv(Dk, m) + n_x;
            const Cplx tb = m * Dk + n_x;
            an = cdiv(cmk(ta.re * psi_n - psi_0, ta.im * psi_n), ta * xi_n - xi_p);
            bn = cdiv(cmk(tb.re * psi_n - psi_0, tb.im * psi_n), tb * xi_n - xi_p);
            psi_m1 = psi_0; psi_0 = psi_n;
            chi_m1 = chi_0; chi_0 = chi_n;
            s_ext += (2.0 * k + 1.0) * (an.re + bn.re);
            s_sca += (2.0 * k + 1.0) * (cabs2(an) + cabs2(bn));
            // asymmetry (Bohren & Huffman eq. 4.62), pairing n-1 with n
            if (k > 1) {
                const double kk = (double)(k - 1);
                s_g += kk * (kk + 2.0) / (kk + 1.0) *
                       (a_prev.re * an.re + a_prev.im * an.im + b_prev.re * bn.re + b_prev.im * bn.im);
            }
            s_g += (2.0 * k + 1.0) / ((double)k * (k + 1.0)) * (an.re * bn.re + an.im * bn.im);
        }
        coef_a[(uint64_t)(k - 1) * n_nodes + i] = an;
        coef_b[(uint64_t)(k - 1) * n_nodes + i] = bn;
        a_prev = an; b_prev = bn;
    }
    I.q_ext = 2.0 / (x * x) * s_ext;
    I.q_sca = 2.0 / (x * x) * s_sca;
    I.g = 4.0 / (x * x * I.q_sca) * s_g;
    info[i] = I;
}

// basis[i][j] = |S1|^2 + |S2|^2 at theta_j for size i; one block per angle.
__global__ void __launch_bounds__(256)
mie_basis_kernel(int n_nodes, int nmax, int n_angles, const MieNodeInfo* __restrict__ info,
                 const Cplx* __restrict__ coef_a, const Cplx* __restrict__ coef_b, double* __restrict__ basis) {
    const int j = blockIdx.x;
    const double theta = (double)j * PI_D / (double)(n_angles - 1);
    const double mu = cos(theta);
    for (int i = threadIdx.x; i < n_nodes; i += blockDim.x) {
        const int nstop = info[i].nstop;
        double pi_prev = 0.0, pi_n = 1.0;
        Cplx S1 = cmk(0.0, 0.0), S2 = cmk(0.0, 0.0);
        for (int k = 1; k <= nstop && k <= nmax; ++k) {
            const double tau_n = (double)k * mu * pi_n - (double)(k + 1) * pi_prev;
            const double f = (2.0 * k + 1.0) / ((double)k * (k + 1.0));
            const Cplx an = coef_a[(uint64_t)(k - 1) * n_nodes + i];
            const Cplx bn = coef_b[(uint64_t)(k - 1) * n_nodes + i];
            S1 = S1 + f * (pi_n * an + tau_n * bn);
            S2 = S2 + f * (tau_n * an + pi_n * bn);
            const double pi_next = ((2.0 * k + 1.0) * mu * pi_n - (double)(k + 1) * pi_prev) / (double)k;
            pi_prev = pi_n; pi_n = pi_next;
        }
        basis[(uint64_t)i * n_angles + j] = cabs2(S1) + cabs2(S2);
    }
}

// --------------------------------------------------------------------------
// Per-set phase function and optics from the basis, then the integer CDF.
// --------------------------------------------------------------------------

__device__ double block_sum(double v, double* sh) {
    const int tid = threadIdx.x, nt = blockDim.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = nt >> 1; off > 0; off >>= 1) {
        if (tid < off) sh[tid] += sh[tid + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Size-averaged Mie intensity of a group of jobs (one optics key, so one
// basis and one angle count): the (jobs x nodes) log-normal weights times
// the (nodes x angles) basis.  A block takes 256 angles of PH_JT jobs, so
// every basis element it reads serves PH_JT jobs; each (job, angle) sum runs
// over the nodes in order.  The blocks of the first angle range also form
// the size-averaged albedo <C_sca>/<C_ext> of their jobs (eq. 11).
constexpr int PH_JT = 8;      // jobs per block
constexpr int PH_NC = 256;    // nodes per weight chunk in LDS

__global__ void __launch_bounds__(256)
mie_phase_kernel(const PhaseJob* __restrict__ jobs, int n_jobs, int n_nodes, const MieNodeInfo* __restrict__ info,
                 const double* __restrict__ basis, uint8_t* tables, SetDesc* descs) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int g0 = blockIdx.y * PH_JT;
    const int nj = min(PH_JT, n_jobs - g0);
    const int na = jobs[g0].n_angles;
    const int j = blockIdx.x * nt + tid;
    __shared__ double s_w[PH_JT][PH_NC];
    __shared__ double s_lnm[PH_JT], s_sig[PH_JT];
    __shared__ double s_red[256];
    if (tid < PH_JT) {
        s_lnm[tid] = tid < nj ? log(jobs[g0 + tid].d_median) : 0.0;
        s_sig[tid] = tid < nj ? jobs[g0 + tid].sigma_ln : 1.0;
    }
    double acc[PH_JT];
#pragma unroll
    for (int t = 0; t < PH_JT; ++t) acc[t] = 0.0;
    for (int c0 = 0; c0 < n_nodes; c0 += PH_NC) {
        const int cn = min(PH_NC, n_nodes - c0);
        __syncthreads();
        // number weights of the truncated log-normal (eq. 21) on the ln d nodes
        for (int e = tid; e < PH_JT * PH_NC; e += nt) {
            const int t = e / PH_NC, i = e % PH_NC;
            double q = 0.0;
            if (t < nj && i < cn) {
                const MieNodeInfo I = info[c0 + i];
                const double z = (I.lnd - s_lnm[t]) / s_sig[t];
                q = I.wq * exp(-0.5 * z * z) / (2.5066282746310002 * s_sig[t]);
            }
            s_w[t][i] = q;
        }
        __syncthreads();
        if (j < na) {
            for (int i = 0; i < cn; ++i) {
                const double b = basis[(uint64_t)(c0 + i) * na + j];
#pragma unroll
                for (int t = 0; t < PH_JT; ++t) acc[t] += s_w[t][i] * b;
            }
        }
    }
    if (j < na) {
        for (int t = 0; t < nj; ++t) {
            double* phase = (double*)(tables + jobs[g0 + t].tab_offset + TableLayout::PHASE);
            phase[j] = acc[t];
        }
    }
    if (blockIdx.x != 0) return;
    for (int t = 0; t < nj; ++t) {
        double sca = 0.0, ext = 0.0;
        for (int i = tid; i < n_nodes; i += nt) {
            const MieNodeInfo I = info[i];
            const double z = (I.lnd - s_lnm[t]) / s_sig[t];
            const double q = I.wq * exp(-0.5 * z * z) / (2.5066282746310002 * s_sig[t]);
            const double x2 = I.x * I.x;
            sca += q * x2 * I.q_sca;
            ext += q * x2 * I.q_ext;
        }
        sca = block_sum(sca, s_red);
        ext = block_sum(ext, s_red);
        if (tid == 0) {
            SetDesc& d = descs[jobs[g0 + t].set];
            const double alb = sca / ext;
            d.albedo = alb;
            d.albedo_f = (float)alb;
            d.albedo_one = alb >= 1.0;
            const double th = floor(alb * 4294967296.0);
            d.thr_albedo = (uint32_t)(th > 4294967295.0 ? 4294967295.0 : (th < 0.0 ? 0.0 : th));
        }
    }
}

__global__ void __launch_bounds__(1024)
phase_cdf_kernel(const PhaseJob* __restrict__ jobs, uint8_t* tables, SetDesc* descs) {
    const PhaseJob J = jobs[blockIdx.x];
    uint8_t* tb = tables + J.tab_offset;
    double* phase = (double*)(tb + TableLayout::PHASE);
    uint32_t* C = (uint32_t*)(tb + TableLayout::CDF);
    uint16_t* cg = (uint16_t*)(tb + TableLayout::CGUIDE);
    __shared__ double s_red[1024];
    __shared__ double s_cell[MAX_ANGLES];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int na = J.n_angles, nc = na - 1;
    SetDesc& d = descs[J.set];
    double* s_ph = s_cell;       // phase values staged here, then replaced by cell masses
    // the phase function sits in the table (caller table, or written by
    // mie_phase_kernel)
    for (int j = tid; j < na; j += nt) s_ph[j] = phase[j];
    __syncthreads();
    // trapezoid cell masses of p sin(theta): q_j = p_j sin(theta_j) first
    double qv[4];
    int nq = 0;
    for (int j = tid; j < na; j += nt) qv[nq++] = s_ph[j] * sin(((double)j * PI_D) / (double)nc);
    __syncthreads();
    nq = 0;
    for (int j = tid; j < na; j += nt) s_ph[j] = qv[nq++];
    __syncthreads();
    double cv[4];
    nq = 0;
    for (int j = tid; j < nc; j += nt) cv[nq++] = 0.5 * (s_ph[j] + s_ph[j + 1]);
    __syncthreads();
    nq = 0;
    for (int j = tid; j < nc; j += nt) s_cell[j] = cv[nq++];
    __syncthreads();
    // exclusive scan in chunks
    const int per = (nc + nt - 1) / nt;
    const int b0 = tid * per, b1 = min(nc, b0 + per);
    double local = 0.0;
    for (int j = b0; j < b1; ++j) local += s_cell[j];
    s_red[tid] = local;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        const double v = tid >= off ? s_red[tid - off] : 0.0;
        __syncthreads();
        s_red[tid] += v;
        __syncthreads();
    }
    const double total = s_red[nt - 1];
    double run = tid > 0 ? s_red[tid - 1] : 0.0;
    double gpart = 0.0;
    const double dth = PI_D / (double)nc;
    __shared__ uint32_t s_C[MAX_ANGLES];
    for (int j = b0; j < b1; ++j) {
        const double F = run / total;
        const double r = floor(F * 4294967296.0 + 0.5);
        const uint32_t cj = j == 0 ? 0u : (uint32_t)(r > 4294967295.0 ? 4294967295.0 : r);
        C[j] = cj;
        s_C[j] = cj;
        run += s_cell[j];
    }
    __syncthreads();
    // exact mean cosine of the sampled law (uniform angle inside each cell)
    for (int j = tid; j < nc; j += nt) {
        const double cj = (double)s_C[j];
        const double cn = j + 1 < nc ? (double)s_C[j + 1] : 4294967296.0;
        const double th0 = ((double)j * PI_D) / (double)nc, th1 = ((double)(j + 1) * PI_D) / (double)nc;
        gpart += (cn - cj) / 4294967296.0 * (sin(th1) - sin(th0)) / dth;
    }
    gpart = block_sum(gpart, s_red);
    // guide: cg[i] = last cell j with C[j] <= i 2^(32 - GUIDE_BITS); every
    // cell writes the entries whose key falls inside it (C is non-decreasing,
    // an empty cell's range is empty and the next cell takes the entries)
    constexpr int SH = 32 - GUIDE_BITS;
    constexpr uint64_t RND = (1ull << SH) - 1ull;
    for (int j = tid; j < nc; j += nt) {
        const uint64_t lo = ((uint64_t)s_C[j] + RND) >> SH;
        const uint64_t hi = j + 1 < nc ? (((uint64_t)s_C[j + 1] + RND) >> SH) : (uint64_t)CDF_GUIDE + 1ull;
        for (uint64_t i = lo; i < hi; ++i) cg[i] = (uint16_t)j;
    }
    if (tid == 0) d.g_mean = gpart;
}

// Ejecta front end (eq. 8-10, 20-21, 27): number-weighted size moments of
// the truncated log-normal on the Mie nodes, and from them the extinction
// optical depth of the whole ejecta and of the slab [v_fs, v_top], the
// size-averaged albedo and efficiency, the Sauter mean diameter and the
// single-scattering model's optical thickness.  One block of 256 threads.
__global__ void __launch_bounds__(256)
ejecta_kernel(int n_nodes, const MieNodeInfo* __restrict__ info, EjectaJob J, double* __restrict__ out) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const double lnm = log(J.d_median);
    double s2 = 0.0, s3 = 0.0, e2 = 0.0, c2 = 0.0;
    for (int i = tid; i < n_nodes; i += 256) {
        const MieNodeInfo I = info[i];
        const double z = (I.lnd - lnm) / J.sigma_ln;
        const double q = I.wq * exp(-0.5 * z * z) / (2.5066282746310002 * J.sigma_ln);
        const double d = exp(I.lnd);
        const double d2 = d * d;
        s2 += q * d2;
        s3 += q * d2 * d;
        e2 += q * d2 * I.q_ext;
        c2 += q * d2 * I.q_sca;
    }
    s2 = block_sum(s2, red);
    s3 = block_sum(s3, red);
    e2 = block_sum(e2, red);
    c2 = block_sum(c2, red);
    if (tid == 0) {
        const double tau_full = 1.5 * J.area_mass * e2 / (J.density * s3);
        const double share = 1.0 - exp(-J.beta * (J.v_top / J.v_fs - 1.0));
        out[0] = tau_full;
        out[1] = tau_full * share;
        out[2] = share;
        out[3] = c2 / e2;
        out[4] = e2 / s2;
        out[5] = s3 / s2;
        out[6] = 1.5 * J.g_back * J.area_mass * e2 / (J.density * s3);
    }
}

// Sets that share another set's tables take its device-computed fields.
__global__ void copy_desc_fields_kernel(SetDesc* d, const int* __restrict__ src, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = src[i];
    if (s == i) return;
    d[i].albedo = d[s].albedo;
    d[i].albedo_f = d[s].albedo_f;
    d[i].thr_albedo = d[s].thr_albedo;
    d[i].albedo_one = d[s].albedo_one;
    d[i].g_mean = d[s].g_mean;
}

// Fill a uint64 range with zeros (graph-safe replacement for a memset).
__global__ void zero_u64_kernel(uint64_t* p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// Copy tally words into callers' device arrays: one block per copy job.
__global__ void copy_jobs_kernel(const CopyJob* __restrict__ jobs, const uint64_t* __restrict__ src) {
    const CopyJob J = jobs[blockIdx.x];
    for (uint64_t i = threadIdx.x; i < J.n_words; i += blockDim.x) J.dst[i] = src[J.src_word + i];
}

}  // namespace pdv

// ---- host launchers ----
namespace pdv {

void launch_layer_tables(hipStream_t s, int n_jobs, const void* jobs, const double* density, uint8_t* tables) {
    if (n_jobs <= 0) return;
    hipLaunchKernelGGL(layer_table_kernel, dim3(n_jobs), dim3(1024), 0, s, (const LayerJob*)jobs, density, tables);
}

void launch_gauss_legendre(hipStream_t s, int n, double* x, double* w) {
    hipLaunchKernelGGL(gauss_legendre_kernel, dim3((n + 127) / 128), dim3(128), 0, s, n, x, w);
}

void launch_mie_nodes(hipStream_t s, int n, const double* gx, const double* gw, double ln_dmin, double ln_dmax,
                      double wavelength, void* info) {
    hipLaunchKernelGGL(mie_nodes_kernel, dim3((n + 127) / 128), dim3(128), 0, s, n, gx, gw, ln_dmin, ln_dmax,
                       wavelength, (MieNodeInfo*)info);
}

void launch_mie_coef(hipStream_t s, int n, int nmax, int nmx_max, double m_re, double m_im, void* info, void* a,
                     void* b, void* dscratch) {
    hipLaunchKernelGGL(mie_coef_kernel, dim3((n + 63) / 64), dim3(64), 0, s, n, nmax, nmx_max, m_re, m_im,
                       (MieNodeInfo*)info, (Cplx*)a, (Cplx*)b, (Cplx*)dscratch);
}

void launch_mie_basis(hipStream_t s, int n, int nmax, int n_angles, const void* info, const void* a, const void* b,
                      double* basis) {
    hipLaunchKernelGGL(mie_basis_kernel, dim3(n_angles), dim3(256), 0, s, n, nmax, n_angles,
                       (const MieNodeInfo*)info, (const Cplx*)a, (const Cplx*)b, basis);
}

// Phase tables of n_jobs jobs: Mie jobs (basis != nullptr; all of one
// optics key) get their size-averaged phase function and albedo first, then
// every job its integer CDF, guide and mean cosine.
void launch_phase_cdf(hipStream_t s, int n_jobs, const void* jobs, int n_nodes, const void* info,
                      const double* basis, uint8_t* tables, SetDesc* descs, int n_angles) {
    if (n_jobs <= 0) return;
    if (basis) {
        const dim3 grid((unsigned)((n_angles + 255) / 256), (unsigned)((n_jobs + PH_JT - 1) / PH_JT));
        hipLaunchKernelGGL(mie_phase_kernel, grid, dim3(256), 0, s, (const PhaseJob*)jobs, n_jobs, n_nodes,
                           (const MieNodeInfo*)info, basis, tables, descs);
    }
    hipLaunchKernelGGL(phase_cdf_kernel, dim3(n_jobs), dim3(1024), 0, s, (const PhaseJob*)jobs, tables, descs);
}

hipError_t launch_ejecta(hipStream_t s, int n_nodes, const void* info, const EjectaJob& J, double* out) {
    hipLaunchKernelGGL(ejecta_kernel, dim3(1), dim3(256), 0, s, n_nodes, (const MieNodeInfo*)info, J, out);
    return hipGetLastError();
}

void launch_copy_desc_fields(hipStream_t s, SetDesc* descs, const int* src, int n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(copy_desc_fields_kernel, dim3((n + 255) / 256), dim3(256), 0, s, descs, src, n);
}

void launch_copy_jobs(hipStream_t s, int n_jobs, const void* jobs, const uint64_t* src) {
    if (n_jobs <= 0) return;
    hipLaunchKernelGGL(copy_jobs_kernel, dim3((unsigned)n_jobs), dim3(256), 0, s, (const CopyJob*)jobs, src);
}

void launch_zero_u64(hipStream_t s, uint64_t* p, uint64_t n) {
    if (n == 0) return;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
}

}  // namespace pdv
