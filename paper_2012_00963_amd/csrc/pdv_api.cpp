// C ABI of libpdv (include/pdv.h): validation, contexts, device memory,
// table building and transport launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "pdv.h"
#include "pdv_internal.h"
#include "pdv_ctx.h"

using namespace pdv;

// ---- kernels (defined in the .hip translation units) ----
namespace pdv {
void launch_layer_tables(hipStream_t s, int n_jobs, const void* jobs, const double* density, uint8_t* tables);
void launch_gauss_legendre(hipStream_t s, int n, double* x, double* w);
void launch_mie_nodes(hipStream_t s, int n, const double* gx, const double* gw, double ln_dmin, double ln_dmax,
                      double wavelength, void* info);
void launch_mie_coef(hipStream_t s, int n, int nmax, int nmx_max, double m_re, double m_im, void* info, void* a,
                     void* b, void* dscratch);
void launch_mie_basis(hipStream_t s, int n, int nmax, int n_angles, const void* info, const void* a, const void* b,
                      double* basis);
void launch_phase_cdf(hipStream_t s, int n_jobs, const void* jobs, int n_nodes, const void* info,
                      const double* basis, uint8_t* tables, SetDesc* descs, int n_angles);
void launch_zero_u64(hipStream_t s, uint64_t* p, uint64_t n);
void launch_copy_jobs(hipStream_t s, int n_jobs, const void* jobs, const uint64_t* src);
void launch_copy_desc_fields(hipStream_t s, SetDesc* descs, const int* src, int n);
int launch_kind_of(const pdv_params* sets, int n);
hipError_t plan_transport(TransportShape& sh, int precision, bool list, int want_bits, int lds_per_block,
                          int lds_per_cu);
SynthPlan synth_plan(int n_frames, int n_samples, uint64_t max_entries);
void launch_frame_ranges(hipStream_t s, int n_frames, uint64_t capacity, const uint64_t* counts, uint64_t* fbeg,
                         uint64_t* fend);
hipError_t launch_synth(hipStream_t s, const SynthPlan& P, int n_frames, int n_samples, const uint64_t* fbeg,
                        const uint64_t* fend, const ListEntry* rec, const float* w, const double* v,
                        const uint32_t* phase, double r_scale, float* partial, float* signal);
hipError_t synth_scratch_init(int device);
float* synth_scratch(int device);
hipError_t launch_stft(hipStream_t s, const float* signal, int n_windows, int nfft, int hop, void* tw, void* tr,
                       float* win, float* map, bool build_tables);
int peak_lds_bytes(int n, int keep);
hipError_t launch_ejecta(hipStream_t s, int n_nodes, const void* info, const EjectaJob& J, double* out);
hipError_t launch_peak(hipStream_t s, int n_spectra, const double* spectra, int n, int keep, const PeakJob& J,
                       double* smoothed, PeakOut* out);
hipError_t launch_transport(hipStream_t s, int precision, bool list, const TransportShape& sh,
                            const SetDesc* descs, const uint8_t* tables, uint64_t* tallies, const WorkItem* items,
                            int n_items, const int* n_items_dev, uint32_t* queue, int persistent, ListEntry* lists,
                            uint64_t* list_counts);
}  // namespace pdv

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
int pdv_ctx::fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    if (code == PDV_EDEVICE) poisoned = true;
    return code;
}

int pdv_ctx::hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return PDV_OK;
    return fail(PDV_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Grow-only pinned host buffer (hipHostMalloc); the stream is synchronised
// before an old buffer is freed.
int pdv_ctx::ensure_pinned(HostPinned& b, size_t bytes, const char* what) {
    if (b.cap >= bytes) return PDV_OK;
    size_t want = std::max(bytes, b.cap + b.cap / 2);
    want = (want + 4095) & ~(size_t)4095;
    if (b.ptr) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_check(e, "synchronize before realloc");
        (void)hipHostFree(b.ptr);
        b.ptr = nullptr;
        b.cap = 0;
    }
    void* p = nullptr;
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PDV_ENOMEM, "%s: hipHostMalloc(%zu) failed: %s", what, want, hipGetErrorString(e));
    }
    b.ptr = p;
    b.cap = want;
    return PDV_OK;
}

int pdv_ctx::ensure(DevBuf& b, size_t bytes, const char* what) {
    if (b.cap >= bytes) return PDV_OK;
    size_t want = std::max(bytes, b.cap + b.cap / 2);
    want = (want + 4095) & ~(size_t)4095;
    if (mem_used - b.cap + want > mem_budget) {
        want = bytes;
        if (mem_used - b.cap + want > mem_budget)
            return fail(PDV_ENOMEM, "%s: %zu bytes exceed the memory budget (%llu used of %llu)", what, bytes,
                        (unsigned long long)mem_used, (unsigned long long)mem_budget);
    }
    if (b.ptr) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_check(e, "synchronize before realloc");
        (void)hipFree(b.ptr);
        mem_used -= b.cap;
        b.ptr = nullptr;
        b.cap = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PDV_ENOMEM, "%s: hipMalloc(%zu) failed: %s", what, want, hipGetErrorString(e));
    }
    b.ptr = p;
    b.cap = want;
    mem_used += want;
    return PDV_OK;
}

static bool is_finite(double v) { return std::isfinite(v); }

namespace pdv {
int validate_params(pdv_ctx* ctx, const pdv_params* p) {
    auto bad = [&](const char* msg) {
        if (ctx) ctx->fail(PDV_EINVAL, "invalid parameters: %s", msg);
        return (int)PDV_EINVAL;
    };
    if (!p) return bad("NULL parameter block");
    if (!is_finite(p->v_bottom) || !is_finite(p->v_top) || p->v_top < p->v_bottom) return bad("need v_top >= v_bottom");
    if (p->n_layers < 1 || p->n_layers > MAX_LAYERS) return bad("n_layers must be in [1, 4096]");
    if (p->density_kind < 0 || p->density_kind > 2) return bad("unknown density_kind");
    if (p->density_kind == PDV_DENSITY_EXP && !(p->v0 > 0.0 && is_finite(p->v0))) return bad("EXP density needs v0 > 0");
    if (p->density_kind == PDV_DENSITY_TABLE) {
        if (!p->density) return bad("TABLE density needs density[n_layers]");
        double tot = 0.0;
        for (int i = 0; i < p->n_layers; ++i) {
            if (!(p->density[i] >= 0.0) || !is_finite(p->density[i])) return bad("density weights must be >= 0");
            tot += p->density[i];
        }
        if (!(tot > 0.0)) return bad("density weights sum to zero");
    }
    if (!(p->tau_total >= 0.0) || !is_finite(p->tau_total) || p->tau_total > 1e4) return bad("tau_total must be in [0, 1e4]");
    if (p->phase_kind < 0 || p->phase_kind > 2) return bad("unknown phase_kind");
    if (p->phase_kind == PDV_PHASE_HG) {
        if (!(std::fabs(p->hg_g) < 1.0)) return bad("|hg_g| must be < 1");
    }
    if (p->phase_kind != PDV_PHASE_HG) {
        if (p->n_angles < 16 || p->n_angles > MAX_ANGLES) return bad("n_angles must be in [16, 4096]");
    }
    if (p->phase_kind != PDV_PHASE_MIE) {
        if (!(p->albedo >= 0.0 && p->albedo <= 1.0)) return bad("albedo must be in [0, 1]");
    }
    if (p->phase_kind == PDV_PHASE_TABLE) {
        if (!p->phase) return bad("TABLE phase needs phase[n_angles]");
        double tot = 0.0;
        for (int i = 0; i < p->n_angles; ++i) {
            if (!(p->phase[i] >= 0.0) || !is_finite(p->phase[i])) return bad("phase values must be >= 0");
            tot += p->phase[i];
        }
        if (!(tot > 0.0)) return bad("phase table is zero");
    }
    if (p->phase_kind == PDV_PHASE_MIE) {
        if (!(p->wavelength > 0.0) || !is_finite(p->wavelength)) return bad("wavelength must be > 0");
        if (!(p->m_re > 0.0) || !(p->m_im >= 0.0) || !is_finite(p->m_re) || !is_finite(p->m_im))
            return bad("refractive index needs m_re > 0, m_im >= 0");
        if (!(p->d_min > 0.0 && p->d_min < p->d_median && p->d_median < p->d_max) || !is_finite(p->d_max))
            return bad("need 0 < d_min < d_median < d_max");
        if (!(p->sigma_ln > 0.0) || !is_finite(p->sigma_ln)) return bad("sigma_ln must be > 0");
        if (p->n_size_nodes < 8 || p->n_size_nodes > 1024) return bad("n_size_nodes must be in [8, 1024]");
        const double xmax = M_PI * p->d_max / p->wavelength;
        if (xmax > 2000.0) return bad("size parameter pi d_max / lambda above 2000");
    }
    if (p->surface_law != PDV_SURFACE_UNIFORM_THETA && p->surface_law != PDV_SURFACE_LAMBERT)
        return bad("unknown surface_law");
    if (!(p->surface_albedo >= 0.0 && p->surface_albedo <= 1.0)) return bad("surface_albedo must be in [0, 1]");
    if (!is_finite(p->v_surface)) return bad("v_surface must be finite");
    if (!(p->cone_half_angle > 0.0 && p->cone_half_angle <= M_PI / 2 + 1e-12))
        return bad("cone_half_angle must be in (0, pi/2]");
    if (p->n_bins < 1 || p->n_bins > MAX_BINS) return bad("n_bins must be in [1, 4096]");
    if (!(p->v_hi > p->v_lo) || !is_finite(p->v_lo) || !is_finite(p->v_hi)) return bad("need v_hi > v_lo");
    if (p->max_orders < 0 || p->max_orders > 100000) return bad("max_orders must be in [0, 100000]");
    if (p->weighting != PDV_WEIGHT_IMPLICIT && p->weighting != PDV_WEIGHT_ANALOG) return bad("unknown weighting");
    if (p->precision != PDV_FP32 && p->precision != PDV_FP64) return bad("precision must be FP32 or FP64");
    if (p->n_packets > 0xFFFFFFFFull) return bad("n_packets must be < 2^32 (fixed-point headroom)");
    if (p->pid_begin + p->n_packets < p->pid_begin) return bad("packet id range overflows");
    return PDV_OK;
}
}  // namespace pdv

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" int pdv_abi_version(void) { return PDV_ABI_VERSION; }

extern "C" int pdv_device_count(int* count) {
    if (!count) return PDV_EINVAL;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *count = 0;
        return PDV_EDEVICE;
    }
    *count = n;
    return PDV_OK;
}

extern "C" int pdv_create(pdv_ctx** out, int device, uint64_t mem_budget, void* hip_stream) {
    if (!out) return PDV_EINVAL;
    pdv_ctx* c = new pdv_ctx();
    *out = c;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) {
        (void)hipGetLastError();
        return c->fail(PDV_EDEVICE, "no HIP device available (%s)", hipGetErrorString(e));
    }
    if (device < 0 || device >= n) return c->fail(PDV_EINVAL, "device %d out of range [0, %d)", device, n);
    c->device = device;
    if (int r = c->hip_check(hipSetDevice(device), "hipSetDevice")) return r;
    hipDeviceProp_t prop;
    if (int r = c->hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties")) return r;
    c->n_cu = prop.multiProcessorCount;
    c->lds_per_block = (int)prop.sharedMemPerBlock;
    c->lds_per_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
    if (c->lds_per_cu < c->lds_per_block) c->lds_per_cu = c->lds_per_block;
    c->arch = prop.gcnArchName;
    size_t free_b = 0, total_b = 0;
    if (int r = c->hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo")) return r;
    c->mem_budget = mem_budget ? mem_budget : (uint64_t)(0.9 * (double)free_b);
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        if (int r = c->hip_check(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "hipStreamCreate"))
            return r;
        c->own_stream = true;
    }
    if (int r = c->hip_check(hipEventCreate(&c->ev_a), "hipEventCreate")) return r;
    if (int r = c->hip_check(hipEventCreate(&c->ev_b), "hipEventCreate")) return r;
    // the allocation-free synthesis entry point's static scratch on this device
    if (int r = c->hip_check(synth_scratch_init(device), "static synthesis scratch")) return r;
    c->ready = true;
    return PDV_OK;
}

extern "C" int pdv_create_host(pdv_ctx** out) {
    if (!out) return PDV_EINVAL;
    pdv_ctx* c = new pdv_ctx();
    c->device = -1;
    c->ready = false;
    c->mem_budget = 1ull << 34;
    *out = c;
    return PDV_OK;
}

extern "C" void pdv_destroy(pdv_ctx* ctx) {
    if (!ctx) return;
    ctx->shutdown_serving();
    if (ctx->ready) {
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
    }
    ctx->release_all();
    if (ctx->ready) {
        if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
        if (ctx->ev_a) (void)hipEventDestroy(ctx->ev_a);
        if (ctx->ev_b) (void)hipEventDestroy(ctx->ev_b);
    }
    delete ctx;
}

bool pdv_ctx::on_device(const void* ptr) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();   // clear the query's error so no later check sees it
        return false;
    }
    return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == device;
}

void pdv_ctx::release_all() {
    DevBuf* all[] = {&descs, &tables, &tallies, &items, &queue, &layer_jobs, &phase_jobs, &density, &lists,
                     &list_counts, &mie_info, &mie_a, &mie_b, &mie_d, &mie_basis, &mie_gx, &mie_gw, &sg_entries,
                     &sg_offsets, &sg_signal, &sg_map, &sg_frames, &sg_partial, &sg_tab, &dup_src, &n_items_dev, &copy_jobs, &pk_in, &pk_smooth, &pk_out, &ej_out};
    if (batch_gexec) (void)hipGraphExecDestroy(batch_gexec);
    batch_gexec = nullptr;
    batch_key = BatchGraphKey{};
    for (DevBuf* b : all) {
        if (b->ptr) (void)hipFree(b->ptr);
        b->ptr = nullptr;
        b->cap = 0;
    }
    for (auto& h : host_pinned) (void)hipHostFree(h.ptr);
    host_pinned.clear();
    for (HostPinned* h : {&tally_pinned, &counts_pinned}) {
        if (h->ptr) (void)hipHostFree(h->ptr);
        *h = HostPinned{};
    }
    mem_used = 0;
    mie_key_valid = false;
    stft_nfft = 0;
}

extern "C" const char* pdv_last_error(const pdv_ctx* ctx) {
    if (!ctx) return "NULL context";
    return ctx->err.c_str();
}

extern "C" int pdv_validate(pdv_ctx* ctx, const pdv_params* p) { return validate_params(ctx, p); }

// ---------------------------------------------------------------------------
// Mie basis (cached per optics key)
// ---------------------------------------------------------------------------
int pdv_ctx::ensure_mie_basis(const pdv_params& p) {
    MieKey k{p.m_re, p.m_im, p.wavelength, p.d_min, p.d_max, p.n_size_nodes, p.n_angles};
    if (mie_key_valid && k == mie_key) return PDV_OK;
    const int n = p.n_size_nodes;
    const double xmax = M_PI * p.d_max / p.wavelength;
    const int nmax = (int)std::floor(xmax + 4.0 * std::cbrt(xmax) + 2.0) + 1;
    const double amx = xmax * std::sqrt(p.m_re * p.m_re + p.m_im * p.m_im);
    const int nmx_max = (int)std::max((double)nmax, std::ceil(amx)) + 17;
    int r;
    if ((r = ensure(mie_gx, sizeof(double) * n, "mie nodes"))) return r;
    if ((r = ensure(mie_gw, sizeof(double) * n, "mie weights"))) return r;
    if ((r = ensure(mie_info, sizeof(MieNodeInfo) * n, "mie node info"))) return r;
    if ((r = ensure(mie_a, 16ull * n * nmax, "mie a_n"))) return r;
    if ((r = ensure(mie_b, 16ull * n * nmax, "mie b_n"))) return r;
    if ((r = ensure(mie_d, 16ull * n * nmax, "mie D_n"))) return r;
    if ((r = ensure(mie_basis, 8ull * n * p.n_angles, "mie basis"))) return r;
    launch_gauss_legendre(stream, n, (double*)mie_gx.ptr, (double*)mie_gw.ptr);
    launch_mie_nodes(stream, n, (const double*)mie_gx.ptr, (const double*)mie_gw.ptr, std::log(p.d_min),
                     std::log(p.d_max), p.wavelength, mie_info.ptr);
    launch_mie_coef(stream, n, nmax, nmx_max, p.m_re, p.m_im, mie_info.ptr, mie_a.ptr, mie_b.ptr, mie_d.ptr);
    launch_mie_basis(stream, n, nmax, p.n_angles, mie_info.ptr, mie_a.ptr, mie_b.ptr, (double*)mie_basis.ptr);
    if ((r = hip_check(hipGetLastError(), "mie basis kernels"))) return r;
    mie_key = k;
    mie_key_valid = true;
    mie_nodes = n;
    return PDV_OK;
}

// ---------------------------------------------------------------------------
// Batch preparation and launch
// ---------------------------------------------------------------------------
// Everything the table kernels read: sets with equal keys get equal tables.
static std::string table_key(const pdv_params& p) {
    std::string k;
    auto put = [&](const void* x, size_t nb) { k.append((const char*)x, nb); };
    put(&p.v_bottom, 8);
    put(&p.v_top, 8);
    put(&p.density_kind, 4);
    put(&p.n_layers, 4);
    put(&p.tau_total, 8);
    if (p.density_kind == PDV_DENSITY_EXP) put(&p.v0, 8);
    if (p.density_kind == PDV_DENSITY_TABLE) put(p.density, 8ull * p.n_layers);
    put(&p.phase_kind, 4);
    if (p.phase_kind == PDV_PHASE_TABLE) {
        put(&p.n_angles, 4);
        put(p.phase, 8ull * p.n_angles);
    }
    if (p.phase_kind == PDV_PHASE_MIE) {
        put(&p.n_angles, 4);
        put(&p.wavelength, 8);
        put(&p.m_re, 8);
        put(&p.m_im, 8);
        put(&p.d_median, 8);
        put(&p.sigma_ln, 8);
        put(&p.d_min, 8);
        put(&p.d_max, 8);
        put(&p.n_size_nodes, 4);
    }
    return k;
}

void pdv::fill_desc(SetDesc& d, const pdv_params& p) {
    std::memset(&d, 0, sizeof d);
    d.v_top = p.v_top;
    d.dzeta = (p.v_top - p.v_bottom) / (double)p.n_layers;
    d.tau_total = p.tau_total;
    d.v_surface = p.v_surface;
    d.surface_albedo = p.surface_albedo;
    d.albedo = p.phase_kind == PDV_PHASE_MIE ? 1.0 : p.albedo;
    d.hg_g = p.phase_kind == PDV_PHASE_HG ? p.hg_g : 0.0;
    d.g_mean = p.phase_kind == PDV_PHASE_HG ? p.hg_g : 0.0;
    d.cos_cone = std::cos(p.cone_half_angle);
    d.v_lo = p.v_lo;
    d.dv = (p.v_hi - p.v_lo) / (double)p.n_bins;
    d.inv_dv = 1.0 / d.dv;
    d.zeta_per_tau = p.tau_total > 0.0 ? (p.v_top - p.v_bottom) / p.tau_total : 0.0;
    d.hg_a = 1.0 + d.hg_g * d.hg_g;
    d.hg_b = 1.0 - d.hg_g * d.hg_g;
    d.hg_c0 = 1.0 - d.hg_g;
    d.hg_c1 = 2.0 * d.hg_g;
    d.hg_inv2g = d.hg_g != 0.0 ? 1.0 / (2.0 * d.hg_g) : 0.0;
    d.lg_scale = p.tau_total > 0.0 ? (double)LAYER_GUIDE / p.tau_total : 0.0;
    d.rev_per_cell = p.phase_kind == PDV_PHASE_HG ? 0.0 : 0.5 / (double)(p.n_angles - 1);
    d.dtheta = p.phase_kind == PDV_PHASE_HG ? 0.0 : 3.14159265358979323846 / (double)(p.n_angles - 1);
    d.uniform_density = p.density_kind == PDV_DENSITY_UNIFORM;
    d.seed = p.seed;
    d.stream = p.stream;
    auto thr = [](double a) {
        double t = std::floor(a * 4294967296.0);
        if (t > 4294967295.0) t = 4294967295.0;
        if (t < 0.0) t = 0.0;
        return (uint32_t)t;
    };
    d.thr_albedo = thr(d.albedo);
    d.thr_surface = thr(p.surface_albedo);
    d.albedo_one = d.albedo >= 1.0;
    d.surface_one = p.surface_albedo >= 1.0;
    d.albedo_f = (float)d.albedo;
    d.surface_albedo_f = (float)p.surface_albedo;
    d.flags = ((p.flags & PDV_FLAG_CLASS_TALLIES) ? SF_CLASS : 0u) | ((p.flags & PDV_FLAG_PEEL) ? SF_PEEL : 0u);
    d.alpha = std::acos(d.cos_cone);
    d.sin2_cone = (1.0 - d.cos_cone) * (1.0 + d.cos_cone);
    d.sin_cone = std::sqrt(d.sin2_cone);
    d.peel_surface_m = p.surface_law == PDV_SURFACE_LAMBERT ? d.sin2_cone : d.alpha / (0.5 * 3.14159265358979323846);
    d.cells_per_rad = p.phase_kind == PDV_PHASE_HG ? 0.0 : (double)(p.n_angles - 1) / 3.14159265358979323846;
    d.n_layers = p.n_layers;
    d.phase_kind = p.phase_kind == PDV_PHASE_HG ? PH_HG : PH_TABLE;
    d.n_cells = p.phase_kind == PDV_PHASE_HG ? 0 : p.n_angles - 1;
    d.surface_law = p.surface_law;
    d.weighting = p.weighting;
    d.max_orders = p.max_orders;
    d.n_bins = p.n_bins;
}

// Kind of a parameter set (KindBits), and of a launch: the specialised kind
// all its FP32 sets share, else KIND_GENERIC.
static int params_kind(const pdv_params& p) {
    return (p.phase_kind != PDV_PHASE_HG ? KB_TABLE : 0) | (p.density_kind == PDV_DENSITY_UNIFORM ? KB_UNIFORM : 0) |
           (p.surface_law == 1 ? KB_LAMBERT : 0) | (p.weighting == 1 ? KB_ANALOG : 0) |
           ((p.flags & PDV_FLAG_CLASS_TALLIES) ? KB_CLASS : 0);
}

int pdv::launch_kind_of(const pdv_params* sets, int n) {
    if (n < 1 || sets[0].precision != PDV_FP32) return KIND_GENERIC;
    const int k0 = params_kind(sets[0]);
    for (int i = 1; i < n; ++i)
        if (params_kind(sets[i]) != k0) return KIND_GENERIC;
    return (k0 == KIND_TABLE_LAYERED || k0 == KIND_HG_UNIFORM) ? k0 : KIND_GENERIC;
}

void pdv_ctx::default_opts(pdv_launch_opts& o, uint64_t total_packets, int n_sets, bool fp64, int kind,
                           bool list, bool peel) const {
    (void)n_sets;
    // measured on the large case: the specialised FP32 kernels run best as
    // two 1024-thread blocks per CU (eight waves per SIMD), the generic FP32
    // kernel as two 768-thread blocks (six waves), FP64 as one 1024-thread
    // block per CU
    // (next-event launches hold six waves per SIMD in every kind)
    const int def_block = fp64 ? 1024 : (kind != KIND_GENERIC && !peel ? 1024 : 768);
    const int def_bpc = fp64 ? 1 : 2;
    if (o.block_size <= 0) o.block_size = tuned.block_size > 0 ? tuned.block_size : def_block;
    if (o.blocks_per_cu <= 0) o.blocks_per_cu = tuned.blocks_per_cu > 0 ? tuned.blocks_per_cu : def_bpc;
    if (o.persistent < 0) o.persistent = tuned.persistent >= 0 ? tuned.persistent : 1;
    if (o.guide_bits == 0) o.guide_bits = tuned.guide_bits;
    // measured: 16 for FP32 spectra (12-16 equal on the large Mie case, 16
    // best by 2 % on the HG slab); 24 when detected
    // packets are also appended to lists (a retire round then also stages
    // its detections: 12 / 24 / 48 / 64 gave 3.57 / 3.03 / 3.15 / 4.54 ms
    // for the 256-frame spectrogram's transport); FP64 is fastest tallying
    // every round
    // 32 for the HG slab kind, whose packets last about 1.5 events (16 / 24 /
    // 32 / 40 / 48 gave 1.34 / 1.24 / 1.24 / 1.24 / 1.27 ms on the 1e8-packet
    // slab once undetected exits stopped contending for one LDS slot)
    if (o.retire_batch == 0)
        o.retire_batch = tuned.retire_batch > 0 ? tuned.retire_batch
                                                : (fp64 ? 1 : (list ? 24 : (kind == KIND_HG_UNIFORM ? 32 : 16)));
    if (o.packets_per_item == 0) {
        // a few large items per block, rounded up so that the item count
        // does not spill into a further round: every item ends with a block
        // barrier that waits for the block's longest packet, and the pull of
        // the last items evens out the blocks' finishing times.  Three per
        // block for spectra (1 / 2 / 3 / 4 / 6 on the 1e8-packet HG slab:
        // 0.94 / 0.97 / 0.91 / 0.99 / 1.01 ms); two for list-writing launches,
        // whose sets (the frames of a spectrogram) each take a block's
        // tables and tallies anew (256 frames of 1e6 packets: 2.13 / 1.98 /
        // 2.05 / 2.01 / 2.06 ms)
        uint64_t grid = (uint64_t)n_cu * (uint64_t)o.blocks_per_cu;
        const uint64_t per_block = list ? 2 : 3;
        uint64_t ppi = (total_packets + per_block * grid - 1) / (per_block * grid);
        ppi = std::max<uint64_t>(ppi, 1024);
        ppi = std::min<uint64_t>(ppi, 1ull << 18);
        o.packets_per_item = tuned.packets_per_item > 0 ? tuned.packets_per_item : ppi;
    }
}

int pdv_ctx::run_batch(const pdv_params* sets, int n, pdv_spectrum_out* outs, const pdv_launch_opts* opts_in,
                       uint64_t list_capacity, bool keep_device, bool defer) {
    if (poisoned) return fail(PDV_EDEVICE, "context poisoned by an earlier device error");
    if (!ready) return fail(PDV_ESTATE, "context not initialised");
    if (!sets || n < 1) return fail(PDV_EINVAL, "need at least one parameter set");
    if (!outs && !keep_device) return fail(PDV_EINVAL, "NULL output array");
    const int precision = sets[0].precision;
    for (int i = 0; i < n; ++i) {
        if (int r = validate_params(this, &sets[i])) return r;
        if (sets[i].precision != precision) return fail(PDV_EINVAL, "all sets of a batch need one precision");
        if (outs && (!outs[i].w_fx || !outs[i].w2_fx)) return fail(PDV_EINVAL, "set %d: NULL w_fx or w2_fx", i);
        if ((sets[i].flags & PDV_FLAG_ACCUMULATE) && (sets[i].flags & PDV_FLAG_DEVICE_OUTPUT))
            return fail(PDV_EINVAL, "set %d: PDV_FLAG_ACCUMULATE applies to host outputs only", i);
        if (sets[i].flags & PDV_FLAG_DEVICE_OUTPUT) {
            if (!outs || list_capacity) return fail(PDV_EINVAL, "set %d: device outputs need a spectrum call", i);
            const bool cls = outs[i].class_fx && (sets[i].flags & PDV_FLAG_CLASS_TALLIES);
            const bool pl = outs[i].peel_fx && (sets[i].flags & PDV_FLAG_PEEL);
            if (!on_device(outs[i].w_fx) || !on_device(outs[i].w2_fx) || (cls && !on_device(outs[i].class_fx)) ||
                (pl && !on_device(outs[i].peel_fx)))
                return fail(PDV_EINVAL, "set %d: PDV_FLAG_DEVICE_OUTPUT needs device arrays on device %d", i, device);
        }
    }
    if (int r = hip_check(hipSetDevice(device), "hipSetDevice")) return r;

    pdv_launch_opts o{0, 0, 0, -1, 0, 0, 0};
    if (opts_in) o = *opts_in;
    uint64_t total = 0;
    for (int i = 0; i < n; ++i) total += sets[i].n_packets;
    const int kind = launch_kind_of(sets, n);
    bool peel = false;
    for (int i = 0; i < n; ++i) peel = peel || (sets[i].flags & PDV_FLAG_PEEL) != 0;
    if (peel && list_capacity) return fail(PDV_EINVAL, "PDV_FLAG_PEEL is for pdv_spectrum and pdv_spectrum_batch only");
    default_opts(o, total, n, precision == PDV_FP64, kind, list_capacity > 0, peel);
    if (o.block_size != 256 && o.block_size != 512 && o.block_size != 768 && o.block_size != 1024)
        return fail(PDV_EINVAL, "block_size must be 256, 512, 768 or 1024");
    if (o.guide_bits != 0 && (o.guide_bits < MIN_GUIDE_BITS || o.guide_bits > GUIDE_BITS))
        return fail(PDV_EINVAL, "guide_bits must be 0 or %d..%d", MIN_GUIDE_BITS, GUIDE_BITS);
    if (o.retire_batch < 1 || o.retire_batch > 64) return fail(PDV_EINVAL, "retire_batch must be 0 or 1..64");
    if (o.persistent != 0 && o.persistent != 1) return fail(PDV_EINVAL, "persistent must be -1, 0 or 1");
    // One set of the tabulated kind and no lists: the persistent launch's
    // waves take work items themselves (kernel mode 2), so no wave waits at
    // an item's end for the block's longest packet; the items are an eighth
    // of a wave's share (unless the caller sets their size), so that the
    // last pulls even out the waves' finishing times.  Large Mie case, items
    // per wave 2 / 4 / 8 / 16: 4.36 / 4.22 / 4.07 / 4.13 ms against 4.18 ms
    // with block items.  A fetch stalls its wave for a global atomic's round
    // trip, which the ~10 events of a packet in a Mie cloud amortise; on the
    // HG slab (1.5 events per packet) the same items cost 0.93 / 0.96 /
    // 1.08 / 1.43 ms against 0.91 ms, so other kinds keep block items.
    const bool wave_items = n == 1 && list_capacity == 0 && o.persistent == 1 && kind == KIND_TABLE_LAYERED;
    if (wave_items && !(opts_in && opts_in->packets_per_item != 0)) {
        const uint64_t waves = (uint64_t)n_cu * (uint64_t)o.blocks_per_cu * (uint64_t)(o.block_size / 64);
        const uint64_t ppi = (total + 8 * waves - 1) / (8 * waves);
        o.packets_per_item = std::min<uint64_t>(std::max<uint64_t>(ppi, 1024), 1ull << 16);
    }
    const int launch_mode = wave_items ? 2 : o.persistent;

    // ---- host-side packing ----
    // Sets whose tables would be identical (same cloud and optics, e.g. the
    // frames of a spectrogram) share one table block; only the first of them
    // runs the table kernels.
    h_desc.assign(n, SetDesc{});
    h_layer.clear();
    h_phase.clear();
    h_density.clear();
    h_src.assign(n, 0);
    std::unordered_map<std::string, int> first_with_key;
    int n_unique = 0;
    uint64_t tally_words_total = 0;
    int max_layers = 1, max_cells = 0, max_bins = 1;
    for (int i = 0; i < n; ++i) {
        const pdv_params& p = sets[i];
        SetDesc& d = h_desc[i];
        fill_desc(d, p);
        auto ins = first_with_key.emplace(table_key(p), i);
        const int src = ins.first->second;
        h_src[i] = src;
        if (src == i) {
            d.tab_offset = (uint64_t)n_unique * TableLayout::BYTES;
            ++n_unique;
            LayerJob L;
            L.v_bottom = p.v_bottom;
            L.v_top = p.v_top;
            L.v0 = p.v0;
            L.tau_total = p.tau_total;
            L.n_layers = p.n_layers;
            L.density_kind = p.density_kind;
            L.tab_offset = d.tab_offset;
            L.density_offset = h_density.size();
            if (p.density_kind == PDV_DENSITY_TABLE)
                h_density.insert(h_density.end(), p.density, p.density + p.n_layers);
            h_layer.push_back(L);
        } else {
            d.tab_offset = h_desc[src].tab_offset;
        }
        d.tally_offset = tally_words_total;
        tally_words_total += tally_words(p.n_bins, d.flags);
        d.list_offset = (uint64_t)i * list_capacity;
        d.list_capacity = list_capacity;
        if (list_capacity) d.flags |= SF_LIST;
        max_layers = std::max(max_layers, p.n_layers);
        max_bins = std::max(max_bins, p.n_bins);
        if (p.phase_kind != PDV_PHASE_HG) max_cells = std::max(max_cells, p.n_angles - 1);
    }
    const int n_layer_jobs = (int)h_layer.size();
    // work items, largest set first
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return sets[a].n_packets > sets[b].n_packets; });
    h_items.clear();
    // wave items: one descriptor of the whole set, which the kernel cuts
    // into n_items equal items itself (a host-built list of the ~65k items
    // of the large case cost ~0.1 ms to build and copy)
    uint64_t n_wave_items = 0;
    if (wave_items) {
        const pdv_params& p = sets[0];
        n_wave_items = (p.n_packets + o.packets_per_item - 1) / o.packets_per_item;
        if (n_wave_items > 0x7fffffffull) return fail(PDV_EINVAL, "too many work items: raise packets_per_item");
        WorkItem w;
        w.set = 0;
        w.pad = 0;
        w.pid_begin = p.pid_begin;
        w.count = p.n_packets;
        if (n_wave_items) h_items.push_back(w);
    } else {
        for (int i : order) {
            const pdv_params& p = sets[i];
            // the set's packets in equal items of at most packets_per_item
            // (sizes differ by one at most: no short remainder that leaves its
            // block idle at the end); items never cross a multiple of 2^32
            // packet ids (a list-writing launch forms detected entries' phase
            // words with one high id word per item)
            const uint64_t n_it = (p.n_packets + o.packets_per_item - 1) / o.packets_per_item;
            const uint64_t even = n_it ? p.n_packets / n_it : 0, extra = n_it ? p.n_packets % n_it : 0;
            uint64_t off = 0;
            for (uint64_t j = 0; j < n_it; ++j) {
                for (uint64_t len = even + (j < extra ? 1 : 0); len > 0;) {
                    WorkItem w;
                    w.set = (uint32_t)i;
                    w.pad = 0;
                    w.pid_begin = p.pid_begin + off;
                    const uint64_t to_wrap = (1ull << 32) - (w.pid_begin & 0xffffffffull);
                    w.count = std::min<uint64_t>(len, to_wrap);
                    h_items.push_back(w);
                    off += w.count;
                    len -= w.count;
                }
            }
        }
    }
    const int n_items = wave_items ? (int)n_wave_items : (int)h_items.size();

    // ---- device buffers ----
    int r;
    if ((r = ensure(descs, sizeof(SetDesc) * n, "set descriptors"))) return r;
    if ((r = ensure(tables, TableLayout::BYTES * (size_t)n_unique, "set tables"))) return r;
    if ((r = ensure(dup_src, sizeof(int) * n, "table sharing map"))) return r;
    if ((r = ensure(tallies, 8ull * tally_words_total, "tallies"))) return r;
    if ((r = ensure(items, sizeof(WorkItem) * std::max<size_t>(1, h_items.size()), "work items"))) return r;
    if ((r = ensure(queue, 256, "queue"))) return r;
    if ((r = ensure(layer_jobs, sizeof(LayerJob) * n, "layer jobs"))) return r;
    if ((r = ensure(phase_jobs, sizeof(PhaseJob) * n, "phase jobs"))) return r;
    if ((r = ensure(density, 8ull * std::max<size_t>(1, h_density.size()), "density staging"))) return r;
    if (list_capacity) {
        if ((r = ensure(lists, sizeof(ListEntry) * list_capacity * (size_t)n, "detected lists"))) return r;
        if ((r = ensure(list_counts, 8ull * n, "list counts"))) return r;
    }

    hipStream_t s = stream;
    auto H2D = [&](void* dst, const void* src, size_t bytes) {
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    if ((r = hip_check(H2D(descs.ptr, h_desc.data(), sizeof(SetDesc) * n), "copy descriptors"))) return r;
    if ((r = hip_check(H2D(layer_jobs.ptr, h_layer.data(), sizeof(LayerJob) * n_layer_jobs), "copy layer jobs")))
        return r;
    if ((r = hip_check(H2D(dup_src.ptr, h_src.data(), sizeof(int) * n), "copy sharing map"))) return r;
    if (!h_density.empty())
        if ((r = hip_check(H2D(density.ptr, h_density.data(), 8 * h_density.size()), "copy densities"))) return r;
    if (n_items)
        if ((r = hip_check(H2D(items.ptr, h_items.data(), sizeof(WorkItem) * h_items.size()), "copy work items")))
            return r;

    // ---- tables ----
    launch_layer_tables(s, n_layer_jobs, layer_jobs.ptr, (const double*)density.ptr, (uint8_t*)tables.ptr);
    // caller phase tables and Mie sets.  Every group's jobs sit in their own
    // range of h_phase (reserved, so it never moves while a copy from it may
    // be in flight) and of the device job array; the host does not wait here
    // (stream order: a group's kernel reads its basis before a later
    // group's basis kernels rewrite it)
    h_phase.reserve(n);
    for (int i = 0; i < n; ++i) {
        const pdv_params& p = sets[i];
        if (h_src[i] != i) continue;
        if (p.phase_kind == PDV_PHASE_TABLE) {
            uint8_t* dst = (uint8_t*)tables.ptr + h_desc[i].tab_offset + TableLayout::PHASE;
            if ((r = hip_check(H2D(dst, p.phase, 8ull * p.n_angles), "copy phase table"))) return r;
            PhaseJob J{1, p.n_angles, 0.0, 0.0, h_desc[i].tab_offset, i, 0};
            h_phase.push_back(J);
        }
    }
    auto launch_group = [&](size_t g0, int n_nodes, const void* info, const double* basis, int n_angles) {
        const size_t ng = h_phase.size() - g0;
        if (ng == 0) return (int)PDV_OK;
        PhaseJob* dj = (PhaseJob*)phase_jobs.ptr + g0;
        if (int e = hip_check(H2D(dj, h_phase.data() + g0, sizeof(PhaseJob) * ng), "copy jobs")) return e;
        launch_phase_cdf(s, (int)ng, dj, n_nodes, info, basis, (uint8_t*)tables.ptr, (SetDesc*)descs.ptr, n_angles);
        return hip_check(hipGetLastError(), "phase table kernels");
    };
    if ((r = launch_group(0, 0, nullptr, nullptr, 0))) return r;
    // Mie sets grouped by optics key (one cached basis at a time)
    std::vector<char> done(n, 0);
    for (int i = 0; i < n; ++i) {
        if (sets[i].phase_kind != PDV_PHASE_MIE || done[i] || h_src[i] != i) continue;
        if ((r = ensure_mie_basis(sets[i]))) return r;
        const size_t g0 = h_phase.size();
        for (int j = i; j < n; ++j) {
            const pdv_params& p = sets[j];
            if (p.phase_kind != PDV_PHASE_MIE || done[j] || h_src[j] != j) continue;
            MieKey k{p.m_re, p.m_im, p.wavelength, p.d_min, p.d_max, p.n_size_nodes, p.n_angles};
            if (!(k == mie_key)) continue;
            PhaseJob J{0, p.n_angles, p.d_median, p.sigma_ln, h_desc[j].tab_offset, j, 0};
            h_phase.push_back(J);
            done[j] = 1;
        }
        if ((r = launch_group(g0, mie_nodes, mie_info.ptr, (const double*)mie_basis.ptr, mie_key.n_angles))) return r;
    }

    if (n_unique < n) launch_copy_desc_fields(s, (SetDesc*)descs.ptr, (const int*)dup_src.ptr, n);

    // ---- transport ----
    launch_zero_u64(s, (uint64_t*)tallies.ptr, tally_words_total);
    if (list_capacity) launch_zero_u64(s, (uint64_t*)list_counts.ptr, (uint64_t)n);
    TransportShape sh;
    sh.block = o.block_size;
    sh.grid = o.persistent ? std::min(n_items, n_cu * o.blocks_per_cu) : n_items;
    if (sh.grid < 1) sh.grid = 1;
    sh.max_layers = max_layers;
    sh.max_cells = max_cells;
    sh.max_bins = max_bins;
    sh.retire_min = o.retire_batch;
    // FP32 sets that all share a specialised kind run that kind's kernel
    sh.kind = kind;
    sh.peel = peel;
    last_kind = sh.kind;
    {
        hipError_t e = plan_transport(sh, precision, list_capacity > 0, o.guide_bits, lds_per_block, lds_per_cu);
        if (e == hipErrorInvalidValue)
            return fail(PDV_EINVAL, "tables need %d bytes of LDS per block (device limit %d)", sh.lds_bytes,
                        lds_per_block);
        if ((r = hip_check(e, "transport launch plan"))) return r;
    }
    last_grid = sh.grid;
    last_block = sh.block;
    last_items = n_items;
    last_guide_bits = sh.guide_bits;
    last_lds = sh.lds_bytes;
    if (o.use_graph && n_items > 0) {
        if ((r = ensure(n_items_dev, 256, "item count"))) return r;
        h_n_items = n_items;
        if ((r = hip_check(H2D(n_items_dev.ptr, &h_n_items, sizeof(int)), "copy item count"))) return r;
    }
    if ((r = hip_check(hipEventRecord(ev_a, s), "event"))) return r;
    if (n_items > 0) {
        if (o.use_graph) {
            if ((r = launch_batch_graph(sh, precision, list_capacity > 0, launch_mode))) return r;
        } else {
            launch_zero_u64(s, (uint64_t*)queue.ptr, 1);
            hipError_t e = launch_transport(s, precision, list_capacity > 0, sh, (const SetDesc*)descs.ptr,
                                            (const uint8_t*)tables.ptr, (uint64_t*)tallies.ptr,
                                            (const WorkItem*)items.ptr, n_items, nullptr, (uint32_t*)queue.ptr,
                                            launch_mode, (ListEntry*)lists.ptr, (uint64_t*)list_counts.ptr);
            if ((r = hip_check(e, "transport launch"))) return r;
        }
    }
    if ((r = hip_check(hipEventRecord(ev_b, s), "event"))) return r;

    // ---- results ----
    // bins of sets with device outputs go device to device into the caller's arrays
    h_copy.clear();
    if (outs) {
        for (int i = 0; i < n; ++i) {
            if (!(sets[i].flags & PDV_FLAG_DEVICE_OUTPUT)) continue;
            const int nb = sets[i].n_bins;
            const uint64_t t0 = h_desc[i].tally_offset;
            h_copy.push_back(CopyJob{t0 + tw_w(nb), (uint64_t)nb, outs[i].w_fx});
            h_copy.push_back(CopyJob{t0 + tw_w2(nb), (uint64_t)nb, outs[i].w2_fx});
            if (outs[i].class_fx && (sets[i].flags & PDV_FLAG_CLASS_TALLIES))
                h_copy.push_back(CopyJob{t0 + tw_class(nb), 2ull * nb, outs[i].class_fx});
            if (outs[i].peel_fx && (sets[i].flags & PDV_FLAG_PEEL))
                h_copy.push_back(CopyJob{t0 + tw_peel(nb, h_desc[i].flags), 2ull * nb, outs[i].peel_fx});
        }
    }
    if (!h_copy.empty()) {
        if ((r = ensure(copy_jobs, sizeof(CopyJob) * h_copy.size(), "output copy jobs"))) return r;
        if ((r = hip_check(H2D(copy_jobs.ptr, h_copy.data(), sizeof(CopyJob) * h_copy.size()), "copy jobs")))
            return r;
        launch_copy_jobs(s, (int)h_copy.size(), copy_jobs.ptr, (const uint64_t*)tallies.ptr);
        if ((r = hip_check(hipGetLastError(), "device output copies"))) return r;
    }
    // tallies and the descriptors the table kernels finished come back
    // through pinned staging (a pageable copy of a 512-set batch's tallies
    // ran at a fraction of the link rate, and a pageable destination would
    // make the host wait for the copy here)
    const size_t tb = 8 * tally_words_total;
    pending_tally_words = tally_words_total;
    if (outs) {       // (a spectrogram without its spectrum keeps the tallies on the device)
        if ((r = ensure_pinned(tally_pinned, tb + sizeof(SetDesc) * n + 8, "tally staging"))) return r;
        uint8_t* ht = (uint8_t*)tally_pinned.ptr;
        if (tb && (r = hip_check(hipMemcpyAsync(ht, tallies.ptr, tb, hipMemcpyDeviceToHost, s), "copy tallies")))
            return r;
        if ((r = hip_check(hipMemcpyAsync(ht + tb, descs.ptr, sizeof(SetDesc) * n, hipMemcpyDeviceToHost, s),
                           "copy descriptors back")))
            return r;
    }
    if (defer) return PDV_OK;
    return finish_batch(sets, n, outs);
}

// Wait for a batch's result copies and unpack them into the outputs.
int pdv_ctx::finish_batch(const pdv_params* sets, int n, pdv_spectrum_out* outs) {
    if (int r = hip_check(hipStreamSynchronize(stream), "transport kernel")) return r;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev_a, ev_b) == hipSuccess) last_kernel_ms = ms;
    if (outs) {
        const uint64_t* ht = (const uint64_t*)tally_pinned.ptr;
        std::memcpy(h_desc.data(), (const uint8_t*)tally_pinned.ptr + 8 * pending_tally_words, sizeof(SetDesc) * n);
        for (int i = 0; i < n; ++i) unpack(sets[i], h_desc[i], ht + h_desc[i].tally_offset, outs[i]);
    }
    return PDV_OK;
}

// The transport launch of a batch as a captured hipGraph: the queue reset
// and the persistent launch, which reads the item count from device memory.
// The graph is kept and replayed while the launch shape and the buffers it
// points to stay the same; any change captures a new one.
int pdv_ctx::launch_batch_graph(const TransportShape& sh, int precision, bool list, int persistent) {
    BatchGraphKey k;
    k.precision = precision;
    k.list = list ? 1 : 0;
    k.persistent = persistent;
    k.grid = sh.grid;
    k.block = sh.block;
    k.lds = sh.lds_bytes;
    k.guide_bits = sh.guide_bits;
    k.retire_min = sh.retire_min;
    k.kind = sh.kind;
    k.peel = sh.peel ? 1 : 0;
    k.max_layers = sh.max_layers;
    k.max_cells = sh.max_cells;
    k.max_bins = sh.max_bins;
    k.ptr[0] = descs.ptr;
    k.ptr[1] = tables.ptr;
    k.ptr[2] = tallies.ptr;
    k.ptr[3] = items.ptr;
    k.ptr[4] = queue.ptr;
    k.ptr[5] = list ? lists.ptr : nullptr;
    k.ptr[6] = list ? list_counts.ptr : nullptr;
    k.ptr[7] = n_items_dev.ptr;
    int r;
    if (!batch_gexec || !(k == batch_key)) {
        if (batch_gexec) {
            (void)hipGraphExecDestroy(batch_gexec);
            batch_gexec = nullptr;
        }
        if ((r = hip_check(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "begin capture")))
            return r;
        launch_zero_u64(stream, (uint64_t*)queue.ptr, 1);
        hipError_t e = launch_transport(stream, precision, list, sh, (const SetDesc*)descs.ptr,
                                        (const uint8_t*)tables.ptr, (uint64_t*)tallies.ptr,
                                        (const WorkItem*)items.ptr, 0, (const int*)n_items_dev.ptr,
                                        (uint32_t*)queue.ptr, persistent, (ListEntry*)lists.ptr,
                                        (uint64_t*)list_counts.ptr);
        hipGraph_t g = nullptr;
        hipError_t ec = hipStreamEndCapture(stream, &g);
        if ((r = hip_check(e, "transport launch (capture)"))) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        if ((r = hip_check(ec, "end capture"))) return r;
        hipError_t ei = hipGraphInstantiate(&batch_gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if ((r = hip_check(ei, "graph instantiate"))) {
            batch_gexec = nullptr;
            return r;
        }
        batch_key = k;
        ++graph_captures;
    }
    ++graph_replays;
    return hip_check(hipGraphLaunch(batch_gexec, stream), "graph launch");
}

void pdv_ctx::unpack(const pdv_params& p, const SetDesc& d, const uint64_t* t, pdv_spectrum_out& o) {
    const int nb = p.n_bins;
    // PDV_FLAG_ACCUMULATE adds to what the outputs hold (a checkpoint of
    // earlier packets); integer sums, so a run resumed in parts equals one run
    const bool acc = (p.flags & PDV_FLAG_ACCUMULATE) != 0;
    auto put = [&](uint64_t* dst, const uint64_t* src, size_t n) {
        if (acc) {
            for (size_t i = 0; i < n; ++i) dst[i] += src[i];
        } else {
            std::memcpy(dst, src, 8 * n);
        }
    };
    auto put1 = [&](uint64_t& dst, uint64_t v) { dst = acc ? dst + v : v; };
    if (!(p.flags & PDV_FLAG_DEVICE_OUTPUT)) {   // device outputs were filled on the device
        put(o.w_fx, t + tw_w(nb), nb);
        put(o.w2_fx, t + tw_w2(nb), nb);
        if (o.class_fx && (p.flags & PDV_FLAG_CLASS_TALLIES)) put(o.class_fx, t + tw_class(nb), 2ull * nb);
        if (o.peel_fx && (p.flags & PDV_FLAG_PEEL)) put(o.peel_fx, t + tw_peel(nb, d.flags), 2ull * nb);
    }
    for (int k = 0; k < PDV_N_SINKS; ++k) put1(o.sinks_fx[k], t[tw_sinks(nb) + k]);
    put1(o.peel_sinks_fx[0], t[tw_sinks(nb) + SK_PEEL_UNDER]);
    put1(o.peel_sinks_fx[1], t[tw_sinks(nb) + SK_PEEL_OVER]);
    const uint64_t* c = t + tw_counts(nb);
    put1(o.counters.packets, c[C_PACKETS]);
    put1(o.counters.collisions, c[C_COLLISIONS]);
    put1(o.counters.surface, c[C_SURFACE]);
    put1(o.counters.exits, c[C_EXITS]);
    put1(o.counters.detected, c[C_DETECTED]);
    o.albedo = d.albedo;
    o.g = d.g_mean;
}

extern "C" int pdv_spectrum(pdv_ctx* ctx, const pdv_params* p, pdv_spectrum_out* out) {
    if (!ctx) return PDV_EINVAL;
    if (ctx->serve) return ctx->fail(PDV_ESTATE, "context is serving: submit requests instead");
    if (!out) return ctx->fail(PDV_EINVAL, "NULL output");
    return ctx->run_batch(p, 1, out, nullptr, 0, false);
}

// Set tables alone: the batch path with no packets builds the tables; the
// realised depth is read back from the set's table block.
extern "C" int pdv_prepare(pdv_ctx* ctx, const pdv_params* p, pdv_table_info* info) {
    if (!ctx) return PDV_EINVAL;
    if (ctx->serve) return ctx->fail(PDV_ESTATE, "context is serving: submit requests instead");
    if (!p || !info) return ctx->fail(PDV_EINVAL, "NULL parameters or output");
    pdv_params q = *p;
    q.n_packets = 0;
    if (q.n_bins < 1 || q.n_bins > MAX_BINS) return ctx->fail(PDV_EINVAL, "n_bins must be 1..%d", MAX_BINS);
    std::vector<uint64_t> w((size_t)q.n_bins), w2((size_t)q.n_bins);
    pdv_spectrum_out out;
    std::memset(&out, 0, sizeof out);
    out.w_fx = w.data();
    out.w2_fx = w2.data();
    if (int r = ctx->run_batch(&q, 1, &out, nullptr, 0, false)) return r;
    const uint8_t* tb = (const uint8_t*)ctx->tables.ptr + ctx->h_desc[0].tab_offset;
    double t64 = 0.0;
    float t32 = 0.f;
    if (int r = ctx->hip_check(hipMemcpy(&t64, tb + TableLayout::T64 + 8ull * q.n_layers, 8, hipMemcpyDeviceToHost),
                               "read layer table"))
        return r;
    if (int r = ctx->hip_check(hipMemcpy(&t32, tb + TableLayout::T32 + 4ull * q.n_layers, 4, hipMemcpyDeviceToHost),
                               "read layer table"))
        return r;
    info->albedo = out.albedo;
    info->g = out.g;
    info->tau_total = t64;
    info->tau_total_f32 = t32;
    info->n_layers = q.n_layers;
    info->n_cells = q.phase_kind == PDV_PHASE_HG ? 0 : q.n_angles - 1;
    return PDV_OK;
}

extern "C" int pdv_spectrum_batch(pdv_ctx* ctx, const pdv_params* sets, int32_t n, pdv_spectrum_out* outs,
                                  const pdv_launch_opts* opts) {
    if (!ctx) return PDV_EINVAL;
    if (ctx->serve) return ctx->fail(PDV_ESTATE, "context is serving: submit requests instead");
    return ctx->run_batch(sets, n, outs, opts, 0, false);
}

extern "C" int pdv_last_launch_kind(const pdv_ctx* ctx) { return ctx ? ctx->last_kind : -1; }

// Timing of the last transport launch (HIP events around the kernel on the
// context stream), its grid and block, for benchmarks.
extern "C" int pdv_last_launch(const pdv_ctx* ctx, float* kernel_ms, int32_t* grid, int32_t* block,
                               int32_t* n_items, int32_t* guide_bits, int32_t* lds_bytes) {
    if (!ctx) return PDV_EINVAL;
    if (kernel_ms) *kernel_ms = ctx->last_kernel_ms;
    if (grid) *grid = ctx->last_grid;
    if (block) *block = ctx->last_block;
    if (n_items) *n_items = ctx->last_items;
    if (guide_bits) *guide_bits = ctx->last_guide_bits;
    if (lds_bytes) *lds_bytes = ctx->last_lds;
    return PDV_OK;
}

// ---------------------------------------------------------------------------
// Stage 2: beat synthesis and spectrogram
// ---------------------------------------------------------------------------
// Entries already on the device (in `lists` when entries == nullptr, else in
// sg_entries); frame k's entries start at entry_begin[k], n_entries[k] of
// them.  Writes the record into sg_signal.
int pdv_ctx::synthesize(int n_frames, const uint64_t* entry_begin, const uint64_t* n_entries,
                        const ListEntry_* entries, double wavelength, double fs, int n_samples) {
    std::vector<uint64_t> fb(2 * (size_t)n_frames);
    uint64_t max_entries = 0;
    for (int k = 0; k < n_frames; ++k) {
        fb[k] = entry_begin[k];
        fb[n_frames + k] = entry_begin[k] + n_entries[k];
        max_entries = std::max<uint64_t>(max_entries, n_entries[k]);
    }
    int r;
    if ((r = ensure(sg_frames, 16ull * n_frames, "synthesis frames"))) return r;
    if ((r = hip_check(hipMemcpyAsync(sg_frames.ptr, fb.data(), 16ull * n_frames, hipMemcpyHostToDevice, stream),
                       "copy frames")))
        return r;
    const uint64_t* d_fb = (const uint64_t*)sg_frames.ptr;
    return synthesize_dev(n_frames, d_fb, d_fb + n_frames, entries, max_entries, wavelength, fs, n_samples);
}

// Frame entry ranges [d_fbeg[k], d_fend[k]) already on the device;
// max_entries bounds every frame's count (it sets the work split).
int pdv_ctx::synthesize_dev(int n_frames, const uint64_t* d_fbeg, const uint64_t* d_fend, const ListEntry_* entries,
                            uint64_t max_entries, double wavelength, double fs, int n_samples) {
    const SynthPlan P = synth_plan(n_frames, n_samples, max_entries);
    int r;
    if ((r = ensure(sg_partial, 4ull * std::max<uint64_t>(1, P.partial_floats), "synthesis partials"))) return r;
    if ((r = ensure(sg_signal, 4ull * std::max(1, n_samples), "beat signal"))) return r;
    const ListEntry* src = entries ? entries : (const ListEntry*)lists.ptr;
    hipError_t e = launch_synth(stream, P, n_frames, n_samples, d_fbeg, d_fend, src, nullptr, nullptr, nullptr,
                                2.0 / (wavelength * fs), (float*)sg_partial.ptr, (float*)sg_signal.ptr);
    return hip_check(e, "beat synthesis kernels");
}

int pdv_ctx::stft(const float* d_signal, int n_samples, int nfft, int hop, int* n_windows) {
    const int nw = n_samples >= nfft ? (n_samples - nfft) / hop + 1 : 0;
    *n_windows = nw;
    const int n = nfft / 2;
    int r;
    const size_t tab_bytes = 8ull * n + 8ull * (n + 1) + 4ull * nfft + 64;
    if ((r = ensure(sg_tab, tab_bytes, "stft tables"))) return r;
    if ((r = ensure(sg_map, 4ull * std::max(1, nw) * (n + 1), "spectrogram map"))) return r;
    uint8_t* base = (uint8_t*)sg_tab.ptr;
    void* tw = base;
    void* tr = base + 8ull * n;
    float* win = (float*)(base + 8ull * n + 8ull * (n + 1));
    const bool build = stft_nfft != nfft;
    hipError_t e = launch_stft(stream, d_signal, nw, nfft, hop, tw, tr, win, (float*)sg_map.ptr, build);
    if ((r = hip_check(e, "stft kernels"))) return r;
    stft_nfft = nfft;
    return PDV_OK;
}

int pdv_spectrogram_internal(pdv_ctx* ctx, const pdv_params* p, const pdv_sg_params* sg, pdv_sg_out* out);

static int check_sg(pdv_ctx* ctx, const pdv_sg_params* sg) {
    if (!sg) return ctx->fail(PDV_EINVAL, "NULL spectrogram parameters");
    if (sg->n_frames < 1 || sg->n_frames > 65535) return ctx->fail(PDV_EINVAL, "n_frames must be in [1, 65535]");
    if (sg->nfft < 256 || sg->nfft > 8192 || (sg->nfft & (sg->nfft - 1)))
        return ctx->fail(PDV_EINVAL, "nfft must be a power of two in [256, 8192]");
    if (sg->hop < 1) return ctx->fail(PDV_EINVAL, "hop must be >= 1");
    if (sg->n_samples < 1 || sg->n_samples > (1 << 28)) return ctx->fail(PDV_EINVAL, "n_samples out of range");
    if (!(sg->fs > 0.0) || !std::isfinite(sg->fs)) return ctx->fail(PDV_EINVAL, "fs must be > 0");
    if (sg->packets_per_frame > 0xFFFFFFFFull) return ctx->fail(PDV_EINVAL, "packets_per_frame must be < 2^32");
    if (sg->list_capacity < 1 || sg->list_capacity > (1ull << 31))
        return ctx->fail(PDV_EINVAL, "list_capacity must be in [1, 2^31]");
    return PDV_OK;
}

extern "C" int pdv_spectrogram(pdv_ctx* ctx, const pdv_params* p, const pdv_sg_params* sg, pdv_sg_out* out) {
    if (!ctx) return PDV_EINVAL;
    if (ctx->serve) return ctx->fail(PDV_ESTATE, "context is serving: submit requests instead");
    return pdv_spectrogram_internal(ctx, p, sg, out);
}

int pdv_spectrogram_internal(pdv_ctx* ctx, const pdv_params* p, const pdv_sg_params* sg, pdv_sg_out* out) {
    if (!out || !out->map) return ctx->fail(PDV_EINVAL, "NULL spectrogram output map");
    if (p && (p->flags & (PDV_FLAG_DEVICE_OUTPUT | PDV_FLAG_PEEL)))
        return ctx->fail(PDV_EINVAL, "PDV_FLAG_DEVICE_OUTPUT and PDV_FLAG_PEEL are for pdv_spectrum and "
                                     "pdv_spectrum_batch only");
    if (int r = check_sg(ctx, sg)) return r;
    if (int r = validate_params(ctx, p)) return r;
    if (!(p->wavelength > 0.0)) return ctx->fail(PDV_EINVAL, "wavelength must be > 0");
    const int F = sg->n_frames;
    std::vector<pdv_params> frames(F, *p);
    for (int k = 0; k < F; ++k) {
        frames[k].stream = p->stream + (uint32_t)k;
        frames[k].n_packets = sg->packets_per_frame;
    }
    const int nb = p->n_bins;
    // per-frame tallies come back only when the summed spectrum is asked for
    const bool want_spec = out->spectrum != nullptr;
    std::vector<uint64_t> W(want_spec ? (size_t)F * nb : 0), W2(want_spec ? (size_t)F * nb : 0);
    std::vector<pdv_spectrum_out> outs(want_spec ? F : 0);
    for (int k = 0; k < (want_spec ? F : 0); ++k) {
        std::memset(&outs[k], 0, sizeof(pdv_spectrum_out));
        outs[k].w_fx = W.data() + (size_t)k * nb;
        outs[k].w2_fx = W2.data() + (size_t)k * nb;
    }
    // transport, frame ranges, synthesis, STFT and the result copies are
    // enqueued back to back; the host waits once, at the end
    if (int r = ctx->run_batch(frames.data(), F, want_spec ? outs.data() : nullptr, nullptr, sg->list_capacity, true,
                               true))
        return r;
    const uint64_t cap = sg->list_capacity;
    if (int r = ctx->ensure(ctx->sg_frames, 16ull * F, "synthesis frames")) return r;
    uint64_t* d_fb = (uint64_t*)ctx->sg_frames.ptr;
    launch_frame_ranges(ctx->stream, F, cap, (const uint64_t*)ctx->list_counts.ptr, d_fb, d_fb + F);
    if (int r = ctx->hip_check(hipGetLastError(), "frame ranges")) return r;
    if (int r = ctx->synthesize_dev(F, d_fb, d_fb + F, nullptr, cap, p->wavelength, sg->fs, sg->n_samples)) return r;
    int nw = 0;
    if (int r = ctx->stft((const float*)ctx->sg_signal.ptr, sg->n_samples, sg->nfft, sg->hop, &nw)) return r;
    if (int r = ctx->ensure_pinned(ctx->counts_pinned, 8ull * F, "list counts")) return r;
    if (int r = ctx->hip_check(hipMemcpyAsync(ctx->counts_pinned.ptr, ctx->list_counts.ptr, 8ull * F,
                                              hipMemcpyDeviceToHost, ctx->stream), "copy list counts"))
        return r;
    const size_t map_floats = (size_t)nw * (sg->nfft / 2 + 1);
    if (map_floats)
        if (int r = ctx->hip_check(hipMemcpyAsync(out->map, ctx->sg_map.ptr, 4 * map_floats, hipMemcpyDeviceToHost,
                                                  ctx->stream), "copy map"))
            return r;
    if (out->signal)
        if (int r = ctx->hip_check(hipMemcpyAsync(out->signal, ctx->sg_signal.ptr, 4ull * sg->n_samples,
                                                  hipMemcpyDeviceToHost, ctx->stream), "copy signal"))
            return r;
    if (int r = ctx->finish_batch(frames.data(), F, want_spec ? outs.data() : nullptr)) return r;
    // detected entries per frame
    std::vector<uint64_t> counts(F), kept(F);
    std::memcpy(counts.data(), ctx->counts_pinned.ptr, 8ull * F);
    int overflow = 0;
    for (int k = 0; k < F; ++k) {
        kept[k] = std::min<uint64_t>(counts[k], cap);
        if (counts[k] > cap) overflow = 1;
    }
    if (out->list_w || out->list_v || out->list_phase) {
        if (!out->list_w || !out->list_v || !out->list_phase || out->list_stride == 0)
            return ctx->fail(PDV_EINVAL, "list output needs list_w, list_v, list_phase and list_stride > 0");
        std::vector<ListEntry> ent((size_t)F * cap);
        if (int r = ctx->hip_check(hipMemcpy(ent.data(), ctx->lists.ptr, sizeof(ListEntry) * ent.size(),
                                             hipMemcpyDeviceToHost), "copy lists"))
            return r;
        for (int k = 0; k < F; ++k) {
            const uint64_t m = std::min<uint64_t>(kept[k], out->list_stride);
            for (uint64_t i = 0; i < m; ++i) {
                const ListEntry& e = ent[(size_t)k * cap + i];
                out->list_w[(size_t)k * out->list_stride + i] = e.w;
                out->list_v[(size_t)k * out->list_stride + i] = e.v;
                out->list_phase[(size_t)k * out->list_stride + i] = e.phase;
            }
        }
    }
    if (out->frame_counts) std::memcpy(out->frame_counts, counts.data(), 8ull * F);
    out->n_windows = nw;
    out->overflow = overflow;
    if (out->spectrum) {
        pdv_spectrum_out* s = out->spectrum;
        if (!s->w_fx || !s->w2_fx) return ctx->fail(PDV_EINVAL, "spectrum output needs w_fx and w2_fx");
        for (int b = 0; b < nb; ++b) {
            uint64_t a = 0, a2 = 0;
            for (int k = 0; k < F; ++k) { a += W[(size_t)k * nb + b]; a2 += W2[(size_t)k * nb + b]; }
            s->w_fx[b] = a;
            s->w2_fx[b] = a2;
        }
        std::memset(s->sinks_fx, 0, sizeof s->sinks_fx);
        std::memset(&s->counters, 0, sizeof s->counters);
        for (int k = 0; k < F; ++k) {
            for (int j = 0; j < PDV_N_SINKS; ++j) s->sinks_fx[j] += outs[k].sinks_fx[j];
            s->counters.packets += outs[k].counters.packets;
            s->counters.collisions += outs[k].counters.collisions;
            s->counters.surface += outs[k].counters.surface;
            s->counters.exits += outs[k].counters.exits;
            s->counters.detected += outs[k].counters.detected;
        }
        s->albedo = outs[0].albedo;
        s->g = outs[0].g;
    }
    return overflow ? PDV_EOVERFLOW : PDV_OK;
}

extern "C" int pdv_beat_synthesize(pdv_ctx* ctx, int32_t n_frames, const uint64_t* offsets, const float* w,
                                   const double* v, const uint32_t* phase_u32, double wavelength, double fs,
                                   int32_t n_samples, float* signal) {
    if (!ctx) return PDV_EINVAL;
    if (ctx->serve) return ctx->fail(PDV_ESTATE, "context is serving: submit requests instead");
    if (ctx->poisoned) return ctx->fail(PDV_EDEVICE, "context poisoned by an earlier device error");
    if (n_frames < 1 || n_frames > SYNTH_MAX_FRAMES || !offsets || !signal)
        return ctx->fail(PDV_EINVAL, "need n_frames in [1, 65535], offsets, signal");
    if (!(wavelength > 0.0) || !(fs > 0.0) || n_samples < 1) return ctx->fail(PDV_EINVAL, "bad wavelength/fs/n_samples");
    const uint64_t total = offsets[n_frames];
    for (int k = 0; k < n_frames; ++k)
        if (offsets[k + 1] < offsets[k]) return ctx->fail(PDV_EINVAL, "offsets must be non-decreasing");
    if (total && (!w || !v || !phase_u32)) return ctx->fail(PDV_EINVAL, "NULL entry arrays");
    if (offsets[0] != 0) return ctx->fail(PDV_EINVAL, "offsets[0] must be 0");
    if (int r = ctx->hip_check(hipSetDevice(ctx->device), "hipSetDevice")) return r;
    std::vector<ListEntry> ent(total);
    for (uint64_t i = 0; i < total; ++i) {
        if (!(w[i] >= 0.0f)) return ctx->fail(PDV_EINVAL, "weights must be >= 0");
        ent[i].w = w[i];
        ent[i].phase = phase_u32[i];
        ent[i].v = v[i];
    }
    int r;
    if ((r = ctx->ensure(ctx->sg_entries, sizeof(ListEntry) * std::max<uint64_t>(1, total), "entries"))) return r;
    if (total)
        if ((r = ctx->hip_check(hipMemcpyAsync(ctx->sg_entries.ptr, ent.data(), sizeof(ListEntry) * total,
                                               hipMemcpyHostToDevice, ctx->stream), "copy entries")))
            return r;
    std::vector<uint64_t> begin(n_frames), cnt(n_frames);
    for (int k = 0; k < n_frames; ++k) {
        begin[k] = offsets[k];
        cnt[k] = offsets[k + 1] - offsets[k];
        if (cnt[k] > 0xFFFFFFFFull) return ctx->fail(PDV_EINVAL, "too many entries in one frame");
    }
    if ((r = ctx->synthesize(n_frames, begin.data(), cnt.data(), (const ListEntry*)ctx->sg_entries.ptr, wavelength,
                             fs, n_samples)))
        return r;
    if ((r = ctx->hip_check(hipMemcpyAsync(signal, ctx->sg_signal.ptr, 4ull * n_samples, hipMemcpyDeviceToHost,
                                           ctx->stream), "copy signal")))
        return r;
    return ctx->hip_check(hipStreamSynchronize(ctx->stream), "beat synthesis");
}

// Allocation-free variant of pdv_beat_synthesize: device inputs and output,
// the groups' partial records in the library's static per-device scratch,
// work enqueued on the context stream without waiting.
extern "C" int pdv_beat_synthesize_static(pdv_ctx* ctx, int32_t n_frames, const uint64_t* offsets, const float* w,
                                          const double* v, const uint32_t* phase_u32, uint64_t max_frame_entries,
                                          double wavelength, double fs, int32_t n_samples, float* signal) {
    if (!ctx) return PDV_EINVAL;
    if (!ctx->ready) return ctx->fail(PDV_ESTATE, "context has no device");
    if (ctx->serve) return ctx->fail(PDV_ESTATE, "context is serving: submit requests instead");
    if (ctx->poisoned) return ctx->fail(PDV_EDEVICE, "context poisoned by an earlier device error");
    if (n_frames < 1 || n_frames > SYNTH_MAX_FRAMES)
        return ctx->fail(PDV_EINVAL, "n_frames must be in [1, 65535]");
    if (n_samples < 1 || n_samples > (1 << 28)) return ctx->fail(PDV_EINVAL, "n_samples must be in [1, 2^28]");
    if (!(wavelength > 0.0) || !(fs > 0.0) || !std::isfinite(wavelength) || !std::isfinite(fs))
        return ctx->fail(PDV_EINVAL, "wavelength and fs must be finite and > 0");
    if (int r = ctx->hip_check(hipSetDevice(ctx->device), "hipSetDevice")) return r;
    if (!offsets || !ctx->on_device(offsets) || !signal || !ctx->on_device(signal))
        return ctx->fail(PDV_EINVAL, "offsets and signal must be device memory of the context's device");
    if (!w || !v || !phase_u32 || !ctx->on_device(w) || !ctx->on_device(v) || !ctx->on_device(phase_u32))
        return ctx->fail(PDV_EINVAL, "w, v and phase_u32 must be device memory of the context's device");
    float* scratch = synth_scratch(ctx->device);
    if (!scratch) return ctx->fail(PDV_ESTATE, "static synthesis scratch not set up on device %d", ctx->device);
    const SynthPlan P = synth_plan(n_frames, n_samples, max_frame_entries);
    if (P.partial_floats > SYNTH_PARTIAL_MAX_FLOATS)
        return ctx->fail(PDV_EINVAL, "partial records of %llu floats exceed the static scratch (%llu)",
                         (unsigned long long)P.partial_floats, (unsigned long long)SYNTH_PARTIAL_MAX_FLOATS);
    hipError_t e = launch_synth(ctx->stream, P, n_frames, n_samples, offsets, offsets + 1, nullptr, w, v, phase_u32,
                                2.0 / (wavelength * fs), scratch, signal);
    return ctx->hip_check(e, "beat synthesis kernels (static scratch)");
}

extern "C" int pdv_stft(pdv_ctx* ctx, const float* signal, int32_t n_samples, int32_t nfft, int32_t hop, float* map,
                        int32_t* n_windows) {
    if (!ctx) return PDV_EINVAL;
    if (ctx->serve) return ctx->fail(PDV_ESTATE, "context is serving: submit requests instead");
    if (ctx->poisoned) return ctx->fail(PDV_EDEVICE, "context poisoned by an earlier device error");
    if (!signal || !map || n_samples < 1) return ctx->fail(PDV_EINVAL, "need signal, map and n_samples >= 1");
    if (nfft < 256 || nfft > 8192 || (nfft & (nfft - 1)))
        return ctx->fail(PDV_EINVAL, "nfft must be a power of two in [256, 8192]");
    if (hop < 1) return ctx->fail(PDV_EINVAL, "hop must be >= 1");
    if (int r = ctx->hip_check(hipSetDevice(ctx->device), "hipSetDevice")) return r;
    int r;
    if ((r = ctx->ensure(ctx->sg_signal, 4ull * n_samples, "signal"))) return r;
    if ((r = ctx->hip_check(hipMemcpyAsync(ctx->sg_signal.ptr, signal, 4ull * n_samples, hipMemcpyHostToDevice,
                                           ctx->stream), "copy signal")))
        return r;
    int nw = 0;
    if ((r = ctx->stft((const float*)ctx->sg_signal.ptr, n_samples, nfft, hop, &nw))) return r;
    if (nw)
        if ((r = ctx->hip_check(hipMemcpyAsync(map, ctx->sg_map.ptr, 4ull * nw * (nfft / 2 + 1),
                                               hipMemcpyDeviceToHost, ctx->stream), "copy map")))
            return r;
    if ((r = ctx->hip_check(hipStreamSynchronize(ctx->stream), "stft"))) return r;
    if (n_windows) *n_windows = nw;
    return PDV_OK;
}

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------
#ifndef PDV_BUILD_ID
#define PDV_BUILD_ID "unknown"
#endif

extern "C" const char* pdv_build_id(void) { return PDV_BUILD_ID; }

extern "C" int pdv_set_launch_defaults(pdv_ctx* ctx, const pdv_launch_opts* o) {
    if (!ctx || !o) return PDV_EINVAL;
    if (o->block_size != 0 && o->block_size != 256 && o->block_size != 512 && o->block_size != 768 &&
        o->block_size != 1024)
        return ctx->fail(PDV_EINVAL, "block_size must be 256, 512, 768 or 1024");
    if (o->blocks_per_cu < 0 || o->blocks_per_cu > 64) return ctx->fail(PDV_EINVAL, "blocks_per_cu out of range");
    if (o->packets_per_item > (1ull << 31)) return ctx->fail(PDV_EINVAL, "packets_per_item out of range");
    if (o->guide_bits != 0 && (o->guide_bits < MIN_GUIDE_BITS || o->guide_bits > GUIDE_BITS))
        return ctx->fail(PDV_EINVAL, "guide_bits must be 0 or %d..%d", MIN_GUIDE_BITS, GUIDE_BITS);
    if (o->retire_batch < 0 || o->retire_batch > 64) return ctx->fail(PDV_EINVAL, "retire_batch must be 0..64");
    ctx->tuned.block_size = o->block_size;
    ctx->tuned.blocks_per_cu = o->blocks_per_cu;
    ctx->tuned.packets_per_item = o->packets_per_item;
    ctx->tuned.persistent = o->persistent;
    ctx->tuned.guide_bits = o->guide_bits;
    ctx->tuned.retire_batch = o->retire_batch;
    return PDV_OK;
}

extern "C" int pdv_autotune(pdv_ctx* ctx, const pdv_params* sets, int32_t n, int32_t repeats,
                            pdv_launch_opts* best, pdv_tune_report* report) {
    if (!ctx) return PDV_EINVAL;
    if (ctx->serve) return ctx->fail(PDV_ESTATE, "context is serving");
    if (!sets || n < 1) return ctx->fail(PDV_EINVAL, "need sets");
    if (repeats < 1) repeats = 3;
    std::vector<std::vector<uint64_t>> W(n), W2(n);
    std::vector<pdv_spectrum_out> outs(n);
    auto run = [&](const pdv_launch_opts& o, float* ms) -> int {
        for (int i = 0; i < n; ++i) {
            W[i].assign(sets[i].n_bins, 0);
            W2[i].assign(sets[i].n_bins, 0);
            std::memset(&outs[i], 0, sizeof(pdv_spectrum_out));
            outs[i].w_fx = W[i].data();
            outs[i].w2_fx = W2[i].data();
        }
        int r = ctx->run_batch(sets, n, outs.data(), &o, 0, false);
        *ms = ctx->last_kernel_ms;
        return r;
    };
    // reference: the current default shape, resolved to explicit values
    pdv_launch_opts def{0, 0, 0, -1, 0, 0, 0};
    {
        uint64_t total = 0;
        for (int i = 0; i < n; ++i) total += sets[i].n_packets;
        ctx->default_opts(def, total, n, sets[0].precision == PDV_FP64, launch_kind_of(sets, n), false);
    }
    float ms = 0;
    if (int r = run(def, &ms)) return r;
    std::vector<std::vector<uint64_t>> refW = W, refW2 = W2;
    std::vector<std::array<uint64_t, PDV_N_SINKS>> refS(n);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < PDV_N_SINKS; ++k) refS[i][k] = outs[i].sinks_fx[k];
    auto median_ms = [&](const pdv_launch_opts& o, double* med, bool* same) -> int {
        std::vector<float> t;
        *same = true;
        for (int rep = 0; rep < repeats; ++rep) {
            if (int r = run(o, &ms)) return r;
            t.push_back(ms);
            for (int i = 0; i < n; ++i) {
                if (W[i] != refW[i] || W2[i] != refW2[i]) *same = false;
                for (int k = 0; k < PDV_N_SINKS; ++k)
                    if (outs[i].sinks_fx[k] != refS[i][k]) *same = false;
            }
        }
        std::sort(t.begin(), t.end());
        *med = t[t.size() / 2];
        return PDV_OK;
    };
    // launch shapes with the default guide resolution, then every guide
    // resolution for the best shape (the table layout stage)
    std::vector<pdv_launch_opts> cands;
    for (int bs : {256, 512, 768, 1024}) {
        for (uint64_t ppi : {1ull << 12, 1ull << 14, 1ull << 16, 1ull << 18}) {
            for (int bpc : {1, 2, 4, 8}) cands.push_back(pdv_launch_opts{bs, bpc, ppi, 1, 0, 0, 0});
            cands.push_back(pdv_launch_opts{bs, 1, ppi, 0, 0, 0, 0});
        }
    }
    double best_ms = 1e300, worst_ms = 0, def_ms = 0;
    bool invariant = true;
    int timed = 1;
    pdv_launch_opts best_o = def;
    {
        bool same = true;
        if (int r = median_ms(def, &def_ms, &same)) return r;
        invariant = invariant && same;
        best_ms = def_ms;
        worst_ms = def_ms;
    }
    auto consider = [&](const pdv_launch_opts& o, bool may_not_fit) -> int {
        double med = 0;
        bool same = true;
        if (int r = median_ms(o, &med, &same)) {
            if (may_not_fit && r == PDV_EINVAL) return PDV_OK;   // staging exceeds the LDS limit
            return r;
        }
        ++timed;
        invariant = invariant && same;
        worst_ms = std::max(worst_ms, med);
        if (med < best_ms) {
            best_ms = med;
            best_o = o;
        }
        return PDV_OK;
    };
    for (const pdv_launch_opts& o : cands)
        if (int r = consider(o, false)) return r;
    {
        pdv_launch_opts base = best_o;
        for (int gb = MIN_GUIDE_BITS; gb <= GUIDE_BITS; ++gb) {
            pdv_launch_opts o = base;
            o.guide_bits = gb;
            if (int r = consider(o, true)) return r;
        }
        base = best_o;
        for (int rb : {4, 8, 12, 24, 32}) {
            pdv_launch_opts o = base;
            o.retire_batch = rb;
            if (int r = consider(o, false)) return r;
        }
    }
    if (report) {
        report->candidates = timed;
        report->invariant = invariant ? 1 : 0;
        report->best_ms = best_ms;
        report->worst_ms = worst_ms;
        report->default_ms = def_ms;
    }
    if (!invariant) return ctx->fail(PDV_EDEVICE, "launch shapes gave different tallies");
    ctx->tuned.block_size = best_o.block_size;
    ctx->tuned.blocks_per_cu = best_o.blocks_per_cu;
    ctx->tuned.packets_per_item = best_o.packets_per_item;
    ctx->tuned.persistent = best_o.persistent;
    ctx->tuned.guide_bits = best_o.guide_bits;
    ctx->tuned.retire_batch = best_o.retire_batch;
    if (best) *best = best_o;
    return PDV_OK;
}

// ---------------------------------------------------------------------------
// Peak analysis
// ---------------------------------------------------------------------------
static_assert(sizeof(pdv_peak_result) == sizeof(PeakOut), "peak result layout");

extern "C" int pdv_peak_analysis(pdv_ctx* ctx, const double* spectra, int32_t n_spectra, const pdv_peak_params* P,
                                 double* smoothed, pdv_peak_result* out) {
    if (!ctx) return PDV_EINVAL;
    if (!spectra || !P || !out || n_spectra < 1) return ctx->fail(PDV_EINVAL, "NULL argument or no spectra");
    if (ctx->poisoned) return ctx->fail(PDV_EDEVICE, "context poisoned by an earlier device error");
    if (!ctx->ready) return ctx->fail(PDV_ESTATE, "context not initialised");
    const int n = P->n_bins, keep = P->keep_modes;
    if (n < 16 || n > 4096) return ctx->fail(PDV_EINVAL, "n_bins must be in [16, 4096]");
    if (keep < 0 || 2 * keep >= n) return ctx->fail(PDV_EINVAL, "keep_modes must be in [0, n_bins/2)");
    if (!(P->v_hi > P->v_lo) || !std::isfinite(P->v_lo) || !std::isfinite(P->v_hi))
        return ctx->fail(PDV_EINVAL, "need v_lo < v_hi");
    if (!(P->v_fs > 0.0) || !std::isfinite(P->v_fs)) return ctx->fail(PDV_EINVAL, "v_fs must be positive");
    PeakJob J{P->v_lo, (P->v_hi - P->v_lo) / (double)n, P->v_fs, P->search_lo, P->search_hi, -1, -1};
    for (int b = 0; b < n; ++b) {
        const double vc = J.v_lo + ((double)b + 0.5) * J.dv;
        if (vc >= J.search_lo && vc < J.search_hi) {
            if (J.wb0 < 0) J.wb0 = b;
            J.wb1 = b;
        }
    }
    if (J.wb0 < 0) return ctx->fail(PDV_EINVAL, "the search window holds no bin centre");
    if (peak_lds_bytes(n, keep) > ctx->lds_per_block)
        return ctx->fail(PDV_EINVAL, "n_bins and keep_modes need more LDS than the device has");
    if (int r = ctx->hip_check(hipSetDevice(ctx->device), "hipSetDevice")) return r;
    const size_t vals = (size_t)n_spectra * (size_t)n;
    int r;
    if ((r = ctx->ensure(ctx->pk_in, 8 * vals, "peak input"))) return r;
    if (smoothed && (r = ctx->ensure(ctx->pk_smooth, 8 * vals, "peak smoothed"))) return r;
    if ((r = ctx->ensure(ctx->pk_out, sizeof(PeakOut) * (size_t)n_spectra, "peak results"))) return r;
    hipStream_t s = ctx->stream;
    if ((r = ctx->hip_check(hipMemcpyAsync(ctx->pk_in.ptr, spectra, 8 * vals, hipMemcpyHostToDevice, s),
                            "copy spectra")))
        return r;
    if ((r = ctx->hip_check(launch_peak(s, n_spectra, (const double*)ctx->pk_in.ptr, n, keep, J,
                                        smoothed ? (double*)ctx->pk_smooth.ptr : nullptr, (PeakOut*)ctx->pk_out.ptr),
                            "peak kernel")))
        return r;
    if ((r = ctx->hip_check(hipMemcpyAsync(out, ctx->pk_out.ptr, sizeof(PeakOut) * (size_t)n_spectra,
                                           hipMemcpyDeviceToHost, s), "copy peak results")))
        return r;
    if (smoothed &&
        (r = ctx->hip_check(hipMemcpyAsync(smoothed, ctx->pk_smooth.ptr, 8 * vals, hipMemcpyDeviceToHost, s),
                            "copy smoothed spectra")))
        return r;
    return ctx->hip_check(hipStreamSynchronize(s), "peak analysis");
}

// ---------------------------------------------------------------------------
// Ejecta front end
// ---------------------------------------------------------------------------
static_assert(sizeof(pdv_ejecta_out) == 7 * sizeof(double), "ejecta output layout");

extern "C" int pdv_ejecta_params(pdv_ctx* ctx, const pdv_ejecta* e, pdv_params* p, pdv_ejecta_out* out) {
    if (!ctx) return PDV_EINVAL;
    if (!e || !p) return ctx->fail(PDV_EINVAL, "NULL ejecta or params");
    if (ctx->poisoned) return ctx->fail(PDV_EDEVICE, "context poisoned by an earlier device error");
    if (!ctx->ready) return ctx->fail(PDV_ESTATE, "context not initialised");
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!pos(e->area_mass) || !pos(e->density) || !pos(e->beta) || !pos(e->v_fs))
        return ctx->fail(PDV_EINVAL, "area_mass, density, beta and v_fs must be positive");
    if (!std::isfinite(e->v_top) || !(e->v_top > e->v_fs)) return ctx->fail(PDV_EINVAL, "need v_top > v_fs");
    if (!std::isfinite(e->g_back) || e->g_back < 0.0) return ctx->fail(PDV_EINVAL, "g_back must be >= 0");
    pdv_params q = *p;
    q.v_bottom = e->v_fs;
    q.v_top = e->v_top;
    q.v_surface = e->v_fs;
    q.density_kind = PDV_DENSITY_EXP;
    q.v0 = e->v_fs / e->beta;
    q.density = nullptr;
    q.phase_kind = PDV_PHASE_MIE;
    q.phase = nullptr;
    q.m_re = e->m_re;
    q.m_im = e->m_im;
    q.wavelength = e->wavelength;
    q.d_median = e->d_median;
    q.sigma_ln = e->sigma_ln;
    q.d_min = e->d_min;
    q.d_max = e->d_max;
    q.n_size_nodes = e->n_size_nodes;
    q.tau_total = 1.0;                    // validated below with the real value
    if (int r = validate_params(ctx, &q)) return r;
    if (int r = ctx->hip_check(hipSetDevice(ctx->device), "hipSetDevice")) return r;
    if (int r = ctx->ensure_mie_basis(q)) return r;
    if (int r = ctx->ensure(ctx->ej_out, 8 * 8, "ejecta results")) return r;
    const EjectaJob J{e->area_mass, e->density, e->beta, e->v_fs, e->v_top, e->d_median, e->sigma_ln, e->g_back};
    double h[7];
    int r;
    if ((r = ctx->hip_check(launch_ejecta(ctx->stream, ctx->mie_nodes, ctx->mie_info.ptr, J, (double*)ctx->ej_out.ptr),
                            "ejecta kernel")))
        return r;
    if ((r = ctx->hip_check(hipMemcpyAsync(h, ctx->ej_out.ptr, sizeof h, hipMemcpyDeviceToHost, ctx->stream),
                            "copy ejecta results")))
        return r;
    if ((r = ctx->hip_check(hipStreamSynchronize(ctx->stream), "ejecta front end"))) return r;
    q.tau_total = h[1];
    if ((r = validate_params(ctx, &q))) return r;
    *p = q;
    if (out) std::memcpy(out, h, sizeof h);
    return PDV_OK;
}
