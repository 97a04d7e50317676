// C ABI of libpdv (include/pdv.h): validation, contexts, device memory,
// table building and transport launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pdv.h"
#include "pdv_internal.h"
#include "pdv_ctx.h"

using namespace pdv;

// ---- kernels (defined in the .hip translation units) ----
namespace pdv {
void launch_layer_tables(hipStream_t s, int n_jobs, const void* jobs, const double* density, uint8_t* tables,
                         SetDesc* descs);
void launch_gauss_legendre(hipStream_t s, int n, double* x, double* w);
void launch_mie_nodes(hipStream_t s, int n, const double* gx, const double* gw, double ln_dmin, double ln_dmax,
                      double wavelength, void* info);
void launch_mie_coef(hipStream_t s, int n, int nmax, int nmx_max, double m_re, double m_im, void* info, void* a,
                     void* b, void* dscratch);
void launch_mie_basis(hipStream_t s, int n, int nmax, int n_angles, const void* info, const void* a, const void* b,
                      double* basis);
void launch_phase_cdf(hipStream_t s, int n_jobs, const void* jobs, int n_nodes, const void* info,
                      const double* basis, uint8_t* tables, SetDesc* descs);
void launch_zero_u64(hipStream_t s, uint64_t* p, uint64_t n);
int transport_lds_bytes(int real_bytes, int max_layers, int max_cells, int max_bins);
hipError_t launch_transport(hipStream_t s, int precision, bool list, int grid, int block, int lds_bytes,
                            const SetDesc* descs, const uint8_t* tables, uint64_t* tallies, const WorkItem* items,
                            int n_items, uint32_t* queue, int persistent, int max_layers, int max_cells,
                            int max_bins, ListEntry* lists, uint64_t* list_counts);
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

static int validate(pdv_ctx* ctx, const pdv_params* p) {
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
    c->ready = true;
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
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->ev_a) (void)hipEventDestroy(ctx->ev_a);
    if (ctx->ev_b) (void)hipEventDestroy(ctx->ev_b);
    delete ctx;
}

void pdv_ctx::release_all() {
    DevBuf* all[] = {&descs, &tables, &tallies, &items, &queue, &layer_jobs, &phase_jobs, &density, &lists,
                     &list_counts, &mie_info, &mie_a, &mie_b, &mie_d, &mie_basis, &mie_gx, &mie_gw, &sg_entries,
                     &sg_offsets, &sg_signal, &sg_map, &sg_frames};
    for (DevBuf* b : all) {
        if (b->ptr) (void)hipFree(b->ptr);
        b->ptr = nullptr;
        b->cap = 0;
    }
    for (auto& h : host_pinned) (void)hipHostFree(h.ptr);
    host_pinned.clear();
    mem_used = 0;
    mie_key_valid = false;
}

extern "C" const char* pdv_last_error(const pdv_ctx* ctx) {
    if (!ctx) return "NULL context";
    return ctx->err.c_str();
}

extern "C" int pdv_validate(pdv_ctx* ctx, const pdv_params* p) { return validate(ctx, p); }

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
static void fill_desc(SetDesc& d, const pdv_params& p) {
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
    d.layer_steps = 13;   // replaced by the table kernels with the exact bound
    d.cdf_steps = 13;
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
    d.flags = (p.flags & PDV_FLAG_CLASS_TALLIES) ? SF_CLASS : 0u;
    d.n_layers = p.n_layers;
    d.phase_kind = p.phase_kind == PDV_PHASE_HG ? PH_HG : PH_TABLE;
    d.n_cells = p.phase_kind == PDV_PHASE_HG ? 0 : p.n_angles - 1;
    d.surface_law = p.surface_law;
    d.weighting = p.weighting;
    d.max_orders = p.max_orders;
    d.n_bins = p.n_bins;
}

void pdv_ctx::default_opts(pdv_launch_opts& o, uint64_t total_packets, int n_sets) const {
    (void)n_sets;
    if (o.block_size <= 0) o.block_size = tuned.block_size > 0 ? tuned.block_size : 512;
    if (o.blocks_per_cu <= 0) o.blocks_per_cu = tuned.blocks_per_cu > 0 ? tuned.blocks_per_cu : 4;
    if (o.persistent < 0) o.persistent = 1;
    if (o.packets_per_item == 0) {
        uint64_t grid = (uint64_t)n_cu * (uint64_t)o.blocks_per_cu;
        uint64_t ppi = total_packets / (grid * 4 + 1);
        ppi = std::max<uint64_t>(ppi, 4096);
        ppi = std::min<uint64_t>(ppi, tuned.packets_per_item > 0 ? tuned.packets_per_item : (1ull << 18));
        o.packets_per_item = ppi;
    }
}

int pdv_ctx::run_batch(const pdv_params* sets, int n, pdv_spectrum_out* outs, const pdv_launch_opts* opts_in,
                       uint64_t list_capacity, bool keep_device) {
    if (poisoned) return fail(PDV_EDEVICE, "context poisoned by an earlier device error");
    if (!ready) return fail(PDV_ESTATE, "context not initialised");
    if (!sets || n < 1) return fail(PDV_EINVAL, "need at least one parameter set");
    if (!outs && !keep_device) return fail(PDV_EINVAL, "NULL output array");
    const int precision = sets[0].precision;
    for (int i = 0; i < n; ++i) {
        if (int r = validate(this, &sets[i])) return r;
        if (sets[i].precision != precision) return fail(PDV_EINVAL, "all sets of a batch need one precision");
        if (outs && (!outs[i].w_fx || !outs[i].w2_fx)) return fail(PDV_EINVAL, "set %d: NULL w_fx or w2_fx", i);
    }
    if (int r = hip_check(hipSetDevice(device), "hipSetDevice")) return r;

    pdv_launch_opts o{0, 0, 0, -1, 0};
    if (opts_in) o = *opts_in;
    uint64_t total = 0;
    for (int i = 0; i < n; ++i) total += sets[i].n_packets;
    default_opts(o, total, n);
    if (o.block_size != 256 && o.block_size != 512 && o.block_size != 1024)
        return fail(PDV_EINVAL, "block_size must be 256, 512 or 1024");

    // ---- host-side packing ----
    h_desc.assign(n, SetDesc{});
    h_layer.assign(n, LayerJob{});
    h_phase.clear();
    h_density.clear();
    uint64_t tally_words_total = 0;
    int max_layers = 1, max_cells = 0, max_bins = 1;
    for (int i = 0; i < n; ++i) {
        const pdv_params& p = sets[i];
        SetDesc& d = h_desc[i];
        fill_desc(d, p);
        d.tab_offset = (uint64_t)i * TableLayout::BYTES;
        d.tally_offset = tally_words_total;
        tally_words_total += tally_words(p.n_bins);
        d.list_offset = (uint64_t)i * list_capacity;
        d.list_capacity = list_capacity;
        if (list_capacity) d.flags |= SF_LIST;
        LayerJob& L = h_layer[i];
        L.v_bottom = p.v_bottom;
        L.v_top = p.v_top;
        L.v0 = p.v0;
        L.tau_total = p.tau_total;
        L.n_layers = p.n_layers;
        L.density_kind = p.density_kind;
        L.tab_offset = d.tab_offset;
        L.density_offset = h_density.size();
        L.set = i;
        L.pad = 0;
        if (p.density_kind == PDV_DENSITY_TABLE) h_density.insert(h_density.end(), p.density, p.density + p.n_layers);
        max_layers = std::max(max_layers, p.n_layers);
        max_bins = std::max(max_bins, p.n_bins);
        if (p.phase_kind != PDV_PHASE_HG) max_cells = std::max(max_cells, p.n_angles - 1);
    }
    // work items, largest set first
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return sets[a].n_packets > sets[b].n_packets; });
    h_items.clear();
    for (int i : order) {
        const pdv_params& p = sets[i];
        for (uint64_t s = 0; s < p.n_packets; s += o.packets_per_item) {
            WorkItem w;
            w.set = (uint32_t)i;
            w.pad = 0;
            w.pid_begin = p.pid_begin + s;
            w.count = std::min<uint64_t>(o.packets_per_item, p.n_packets - s);
            h_items.push_back(w);
        }
    }
    const int n_items = (int)h_items.size();

    // ---- device buffers ----
    int r;
    if ((r = ensure(descs, sizeof(SetDesc) * n, "set descriptors"))) return r;
    if ((r = ensure(tables, TableLayout::BYTES * (size_t)n, "set tables"))) return r;
    if ((r = ensure(tallies, 8ull * tally_words_total, "tallies"))) return r;
    if ((r = ensure(items, sizeof(WorkItem) * std::max(1, n_items), "work items"))) return r;
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
    if ((r = hip_check(H2D(layer_jobs.ptr, h_layer.data(), sizeof(LayerJob) * n), "copy layer jobs"))) return r;
    if (!h_density.empty())
        if ((r = hip_check(H2D(density.ptr, h_density.data(), 8 * h_density.size()), "copy densities"))) return r;
    if (n_items)
        if ((r = hip_check(H2D(items.ptr, h_items.data(), sizeof(WorkItem) * n_items), "copy work items"))) return r;

    // ---- tables ----
    launch_layer_tables(s, n, layer_jobs.ptr, (const double*)density.ptr, (uint8_t*)tables.ptr,
                        (SetDesc*)descs.ptr);
    // caller phase tables and Mie sets
    for (int i = 0; i < n; ++i) {
        const pdv_params& p = sets[i];
        if (p.phase_kind == PDV_PHASE_TABLE) {
            uint8_t* dst = (uint8_t*)tables.ptr + h_desc[i].tab_offset + TableLayout::PHASE;
            if ((r = hip_check(H2D(dst, p.phase, 8ull * p.n_angles), "copy phase table"))) return r;
            PhaseJob J{1, p.n_angles, 0.0, 0.0, h_desc[i].tab_offset, i, 0};
            h_phase.push_back(J);
        }
    }
    if (!h_phase.empty()) {
        if ((r = hip_check(H2D(phase_jobs.ptr, h_phase.data(), sizeof(PhaseJob) * h_phase.size()), "copy jobs")))
            return r;
        launch_phase_cdf(s, (int)h_phase.size(), phase_jobs.ptr, 0, nullptr, nullptr, (uint8_t*)tables.ptr,
                         (SetDesc*)descs.ptr);
        if ((r = hip_check(hipStreamSynchronize(s), "table kernels"))) return r;
    }
    // Mie sets grouped by optics key (one cached basis at a time)
    std::vector<char> done(n, 0);
    for (int i = 0; i < n; ++i) {
        if (sets[i].phase_kind != PDV_PHASE_MIE || done[i]) continue;
        if ((r = ensure_mie_basis(sets[i]))) return r;
        h_phase.clear();
        for (int j = i; j < n; ++j) {
            const pdv_params& p = sets[j];
            if (p.phase_kind != PDV_PHASE_MIE || done[j]) continue;
            MieKey k{p.m_re, p.m_im, p.wavelength, p.d_min, p.d_max, p.n_size_nodes, p.n_angles};
            if (!(k == mie_key)) continue;
            PhaseJob J{0, p.n_angles, p.d_median, p.sigma_ln, h_desc[j].tab_offset, j, 0};
            h_phase.push_back(J);
            done[j] = 1;
        }
        if ((r = hip_check(H2D(phase_jobs.ptr, h_phase.data(), sizeof(PhaseJob) * h_phase.size()), "copy jobs")))
            return r;
        launch_phase_cdf(s, (int)h_phase.size(), phase_jobs.ptr, mie_nodes, mie_info.ptr,
                         (const double*)mie_basis.ptr, (uint8_t*)tables.ptr, (SetDesc*)descs.ptr);
        if ((r = hip_check(hipStreamSynchronize(s), "mie phase kernels"))) return r;
    }

    // ---- transport ----
    launch_zero_u64(s, (uint64_t*)tallies.ptr, tally_words_total);
    launch_zero_u64(s, (uint64_t*)queue.ptr, 1);
    if (list_capacity) launch_zero_u64(s, (uint64_t*)list_counts.ptr, (uint64_t)n);
    const int lds = transport_lds_bytes(precision == PDV_FP64 ? 8 : 4, max_layers, max_cells, max_bins);
    if (lds > 64 * 1024) return fail(PDV_EINVAL, "tables need %d bytes of LDS per block (limit 65536)", lds);
    int grid = o.persistent ? std::min(n_items, n_cu * o.blocks_per_cu) : n_items;
    if (grid < 1) grid = 1;
    last_grid = grid;
    last_block = o.block_size;
    last_items = n_items;
    if ((r = hip_check(hipEventRecord(ev_a, s), "event"))) return r;
    if (n_items > 0) {
        hipError_t e = launch_transport(s, precision, list_capacity > 0, grid, o.block_size, lds,
                                        (const SetDesc*)descs.ptr, (const uint8_t*)tables.ptr,
                                        (uint64_t*)tallies.ptr, (const WorkItem*)items.ptr, n_items,
                                        (uint32_t*)queue.ptr, o.persistent, max_layers, max_cells, max_bins,
                                        (ListEntry*)lists.ptr, (uint64_t*)list_counts.ptr);
        if ((r = hip_check(e, "transport launch"))) return r;
    }
    if ((r = hip_check(hipEventRecord(ev_b, s), "event"))) return r;

    // ---- results ----
    h_tally.resize(tally_words_total);
    if ((r = hip_check(hipMemcpyAsync(h_tally.data(), tallies.ptr, 8 * tally_words_total, hipMemcpyDeviceToHost, s),
                       "copy tallies")))
        return r;
    if ((r = hip_check(hipMemcpyAsync(h_desc.data(), descs.ptr, sizeof(SetDesc) * n, hipMemcpyDeviceToHost, s),
                       "copy descriptors back")))
        return r;
    if ((r = hip_check(hipStreamSynchronize(s), "transport kernel"))) return r;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev_a, ev_b) == hipSuccess) last_kernel_ms = ms;
    if (outs) {
        for (int i = 0; i < n; ++i) unpack(sets[i], h_desc[i], h_tally.data() + h_desc[i].tally_offset, outs[i]);
    }
    return PDV_OK;
}

void pdv_ctx::unpack(const pdv_params& p, const SetDesc& d, const uint64_t* t, pdv_spectrum_out& o) {
    const int nb = p.n_bins;
    std::memcpy(o.w_fx, t + tw_w(nb), 8ull * nb);
    std::memcpy(o.w2_fx, t + tw_w2(nb), 8ull * nb);
    if (o.class_fx && (p.flags & PDV_FLAG_CLASS_TALLIES)) std::memcpy(o.class_fx, t + tw_class(nb), 16ull * nb);
    for (int k = 0; k < PDV_N_SINKS; ++k) o.sinks_fx[k] = t[tw_sinks(nb) + k];
    const uint64_t* c = t + tw_counts(nb);
    o.counters.packets = c[C_PACKETS];
    o.counters.collisions = c[C_COLLISIONS];
    o.counters.surface = c[C_SURFACE];
    o.counters.exits = c[C_EXITS];
    o.counters.detected = c[C_DETECTED];
    o.albedo = d.albedo;
    o.g = d.g_mean;
}

extern "C" int pdv_spectrum(pdv_ctx* ctx, const pdv_params* p, pdv_spectrum_out* out) {
    if (!ctx) return PDV_EINVAL;
    if (!out) return ctx->fail(PDV_EINVAL, "NULL output");
    return ctx->run_batch(p, 1, out, nullptr, 0, false);
}

extern "C" int pdv_spectrum_batch(pdv_ctx* ctx, const pdv_params* sets, int32_t n, pdv_spectrum_out* outs,
                                  const pdv_launch_opts* opts) {
    if (!ctx) return PDV_EINVAL;
    return ctx->run_batch(sets, n, outs, opts, 0, false);
}

// Timing of the last transport launch (HIP events around the kernel on the
// context stream), its grid and block, for benchmarks.
extern "C" int pdv_last_launch(const pdv_ctx* ctx, float* kernel_ms, int32_t* grid, int32_t* block,
                               int32_t* n_items) {
    if (!ctx) return PDV_EINVAL;
    if (kernel_ms) *kernel_ms = ctx->last_kernel_ms;
    if (grid) *grid = ctx->last_grid;
    if (block) *block = ctx->last_block;
    if (n_items) *n_items = ctx->last_items;
    return PDV_OK;
}
