// Serving engine: continuous batching of spectrum requests on one GPU.
//
// Clients submit requests (a parameter set, optionally a spectrogram) from
// any thread; one scheduler thread owns the device.  Every iteration it
//   1. admits waiting requests in arrival order while a slot and enough of
//      the memory budget are free (a request larger than the whole budget is
//      refused at submission),
//   2. builds the device tables of the newly admitted requests into their
//      slots (layer depths, Mie phase CDF from the resident Mie basis),
//   3. issues the next slice of packets of every active request as work
//      items of one persistent transport launch (replayed from a captured
//      hipGraph when enabled),
//   4. retires requests whose packets are all transported: copies their
//      tallies to the caller's buffers (one batched device-to-host copy per
//      iteration) and stamps the latency (submission -> result on the host).
// A request that also asks for a spectrogram is handed, once its spectrum
// is done, to a spectrogram worker thread that owns a second context with
// its own stream, so its frame transport, beat synthesis and STFT overlap
// on the device with the scheduler's next iterations instead of stalling
// them.  Requests that arrive while an iteration runs join the next one, so
// their work overlaps on the device with older requests.  Tallies are integer sums
// over the same (seed, stream, packet id) random streams whatever the slicing,
// so a result is bitwise the same alone and in any mix.
//
// An executor interface separates the scheduler from the device: the HIP
// executor runs the kernels; a host executor (for scheduler tests without a
// GPU) completes items arithmetically, can be slowed down and can fail at a
// chosen iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "pdv_ctx.h"

using namespace pdv;

int pdv_spectrogram_internal(pdv_ctx* ctx, const pdv_params* p, const pdv_sg_params* sg, pdv_sg_out* out);

namespace pdv {
int validate_params(pdv_ctx* ctx, const pdv_params* p);
void fill_desc(SetDesc& d, const pdv_params& p);
void launch_layer_tables(hipStream_t s, int n_jobs, const void* jobs, const double* density, uint8_t* tables);
void launch_phase_cdf(hipStream_t s, int n_jobs, const void* jobs, int n_nodes, const void* info,
                      const double* basis, uint8_t* tables, SetDesc* descs, int n_angles);
void launch_zero_u64(hipStream_t s, uint64_t* p, uint64_t n);
hipError_t plan_transport(TransportShape& sh, int precision, bool list, int want_bits, int lds_per_block,
                          int lds_per_cu);
int launch_kind_of(const pdv_params* sets, int n);
hipError_t launch_transport_dev(hipStream_t s, int precision, const TransportShape& sh, const SetDesc* descs,
                                const uint8_t* tables, uint64_t* tallies, const WorkItem* items,
                                const int* n_items_dev, uint32_t* queue);
}  // namespace pdv

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
    uint64_t ticket = 0;
    pdv_params p{};
    std::vector<double> density, phase;
    bool want_sg = false;
    pdv_sg_params sg{};
    pdv_spectrum_out* out = nullptr;
    pdv_sg_out* sg_out = nullptr;
    int status = PDV_PENDING;          // final status once != PDV_PENDING
    bool cancel = false;
    bool waited = false;               // counted once in admission waits
    int slot = -1;
    uint64_t issued = 0;               // packets handed to launches
    uint64_t footprint = 0;            // bytes of device memory while active
    double t_submit = 0, t_admit = 0, t_done = 0;
};

uint64_t slot_tally_words(int max_bins) { return tally_words(max_bins, SF_CLASS); }

}  // namespace

// ---------------------------------------------------------------------------
// executors
// ---------------------------------------------------------------------------
struct Executor {
    virtual ~Executor() = default;
    virtual int init() = 0;
    virtual int prepare(const std::vector<Req*>& admitted) = 0;
    // finishing: requests whose last packets are in this launch (their
    // results may be copied back right after it); kind: the kernel kind
    // every set of the launch shares (KIND_GENERIC for a mix)
    virtual int run(const std::vector<WorkItem>& items, const std::vector<Req*>& finishing, int kind) = 0;
    // copy the finished requests' results to their callers (st[i] per request)
    virtual int collect(const std::vector<Req*>& done, std::vector<int>& st) = 0;
    virtual const char* error() const = 0;
};

struct ServeEngine {
    pdv_ctx* ctx = nullptr;
    pdv_serve_opts opts{};
    std::unique_ptr<Executor> exec;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Req>> pending;
    std::vector<std::shared_ptr<Req>> active;
    std::unordered_map<uint64_t, std::shared_ptr<Req>> by_ticket;
    std::vector<int> free_slots;
    std::vector<int> slot_bins;        // n_bins of the request holding each slot
    uint64_t mem_in_use = 0;
    uint64_t next_ticket = 1;
    bool stopping = false, drain = true, failed = false;
    std::string fail_msg;
    std::thread th;
    // statistics
    uint64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_cancelled = 0, n_iterations = 0;
    uint64_t n_packets = 0, n_events = 0;
    uint64_t n_admit_waits = 0;
    std::vector<double> latencies_ms, queue_ms;
    double t_start = 0, busy_s = 0;
    double prepare_s = 0, launch_s = 0, collect_s = 0, sg_s = 0;
    // spectrogram worker: its own context (device buffers, stream)
    std::vector<pdv_ctx*> sg_ctx;        // one context (buffers, Mie basis, stream) per worker
    std::deque<std::shared_ptr<Req>> sg_queue;
    std::condition_variable cv_sg;
    bool sg_stop = false;
    std::vector<std::thread> sg_th;

    void loop();
    void sg_loop(int worker);
    void join_all();
    // final status of a request (caller holds mu)
    void finish(const std::shared_ptr<Req>& q, int st);
    uint64_t footprint(const Req& r) const;
    int active_bins(int slot) const;
};

// HIP executor: slots of a fixed-capacity device arena.
struct HipExecutor : Executor {
    ServeEngine* E;
    pdv_ctx* ctx;
    DevBuf descs, tables, tallies, items, nitems, queue, layer_jobs, phase_jobs, density;
    WorkItem* h_items = nullptr;     // pinned staging for graph replays
    int* h_nitems = nullptr;
    SetDesc* h_desc = nullptr;       // pinned staging: descriptors per slot (in and out)
    LayerJob* h_lj = nullptr;        // pinned staging: layer jobs of one iteration
    PhaseJob* h_pj = nullptr;        // pinned staging: phase jobs of one iteration
    uint64_t* h_tally = nullptr;     // pinned staging: tally blocks per slot
    int max_items = 0;
    // One launch shape and one captured graph per kernel kind: the generic
    // kernel (any mix of requests) and the two specialised FP32 kinds, which
    // give bit-identical tallies.  512-thread blocks, as many per CU as the
    // kernel's occupancy keeps resident (four at eight waves per SIMD, three
    // at six, two at four).
    static constexpr int N_KIND = 3;
    TransportShape shape_k[N_KIND];
    hipGraphExec_t gexec_k[N_KIND] = {};
    hipGraph_t graph_k[N_KIND] = {};
    static int kind_index(int kind) { return kind == KIND_TABLE_LAYERED ? 1 : (kind == KIND_HG_UNIFORM ? 2 : 0); }
    std::string err;

    explicit HipExecutor(ServeEngine* e) : E(e), ctx(e->ctx) {}
    ~HipExecutor() override {
        for (int k = 0; k < N_KIND; ++k) {
            if (gexec_k[k]) (void)hipGraphExecDestroy(gexec_k[k]);
            if (graph_k[k]) (void)hipGraphDestroy(graph_k[k]);
        }
        DevBuf* all[] = {&descs, &tables, &tallies, &items, &nitems, &queue, &layer_jobs, &phase_jobs, &density};
        for (DevBuf* b : all)
            if (b->ptr) {
                (void)hipFree(b->ptr);
                ctx->mem_used -= b->cap;
            }
        void* pinned[] = {h_items, h_nitems, h_desc, h_lj, h_pj, h_tally};
        for (void* h : pinned)
            if (h) (void)hipHostFree(h);
    }
    const char* error() const override { return err.c_str(); }
    int hipfail(hipError_t e, const char* what) {
        if (e == hipSuccess) return PDV_OK;
        err = std::string(what) + ": " + hipGetErrorString(e);
        return PDV_EDEVICE;
    }
    int init() override {
        const int S = E->opts.max_active;
        int r;
        if ((r = ctx->ensure(descs, sizeof(SetDesc) * S, "serve descriptors"))) return r;
        if ((r = ctx->ensure(tables, TableLayout::BYTES * (size_t)S, "serve tables"))) return r;
        if ((r = ctx->ensure(tallies, 8ull * slot_tally_words(E->opts.max_bins) * S, "serve tallies"))) return r;
        max_items = E->opts.max_items;
        if ((r = ctx->ensure(items, sizeof(WorkItem) * max_items, "serve items"))) return r;
        if ((r = ctx->ensure(nitems, 256, "serve item count"))) return r;
        if ((r = ctx->ensure(queue, 256, "serve queue"))) return r;
        if ((r = ctx->ensure(layer_jobs, sizeof(LayerJob) * S, "serve layer jobs"))) return r;
        if ((r = ctx->ensure(phase_jobs, sizeof(PhaseJob) * S, "serve phase jobs"))) return r;
        if ((r = hipfail(hipHostMalloc((void**)&h_items, sizeof(WorkItem) * max_items, hipHostMallocDefault),
                         "pinned items"))) return r;
        if ((r = hipfail(hipHostMalloc((void**)&h_nitems, 256, hipHostMallocDefault), "pinned count"))) return r;
        if ((r = hipfail(hipHostMalloc((void**)&h_desc, sizeof(SetDesc) * S, hipHostMallocDefault),
                         "pinned descriptors"))) return r;
        if ((r = hipfail(hipHostMalloc((void**)&h_lj, sizeof(LayerJob) * S, hipHostMallocDefault),
                         "pinned layer jobs"))) return r;
        if ((r = hipfail(hipHostMalloc((void**)&h_pj, sizeof(PhaseJob) * S, hipHostMallocDefault),
                         "pinned phase jobs"))) return r;
        if ((r = hipfail(hipHostMalloc((void**)&h_tally, 8ull * slot_tally_words(E->opts.max_bins) * S,
                                       hipHostMallocDefault), "pinned tallies"))) return r;
        const bool fp64 = E->opts.precision == PDV_FP64;
        const int kinds[N_KIND] = {KIND_GENERIC, KIND_TABLE_LAYERED, KIND_HG_UNIFORM};
        for (int k = 0; k < (fp64 ? 1 : N_KIND); ++k) {
            TransportShape& sh = shape_k[k];
            sh.kind = kinds[k];
            sh.block = 512;
            sh.grid = ctx->n_cu * (fp64 ? 2 : (k == 0 ? 3 : 4));
            sh.max_layers = E->opts.max_layers;
            sh.max_cells = E->opts.max_angles - 1;
            sh.max_bins = E->opts.max_bins;
            sh.retire_min = fp64 ? 1 : 12;
            hipError_t e = plan_transport(sh, E->opts.precision, false, 0, ctx->lds_per_block, ctx->lds_per_cu);
            if (e == hipErrorInvalidValue) {
                err = "serving limits need more LDS per block than the device has";
                return PDV_EINVAL;
            }
            if ((r = hipfail(e, "transport launch plan"))) return r;
        }
        return PDV_OK;
    }
    // Tables of the newly admitted requests, all enqueued on the context
    // stream from pinned staging; the transport launch that follows on the
    // same stream sees them complete.
    int prepare(const std::vector<Req*>& adm) override {
        if (adm.empty()) return PDV_OK;
        hipStream_t s = ctx->stream;
        std::vector<double> dens;
        const int na = (int)adm.size();
        for (int i = 0; i < na; ++i) {
            const Req* q = adm[i];
            SetDesc& d = h_desc[q->slot];
            fill_desc(d, q->p);
            d.tab_offset = (uint64_t)q->slot * TableLayout::BYTES;
            d.tally_offset = (uint64_t)q->slot * slot_tally_words(E->opts.max_bins);
            h_lj[i] = LayerJob{q->p.v_bottom, q->p.v_top, q->p.v0, q->p.tau_total, q->p.n_layers,
                               q->p.density_kind, d.tab_offset, dens.size()};
            if (q->p.density_kind == PDV_DENSITY_TABLE) dens.insert(dens.end(), q->density.begin(), q->density.end());
        }
        int r;
        if ((r = ctx->ensure(density, 8 * std::max<size_t>(1, dens.size()), "serve density"))) return r;
        for (int i = 0; i < na; ++i)
            if ((r = hipfail(hipMemcpyAsync((SetDesc*)descs.ptr + adm[i]->slot, h_desc + adm[i]->slot,
                                            sizeof(SetDesc), hipMemcpyHostToDevice, s), "copy descriptor")))
                return r;
        if ((r = hipfail(hipMemcpyAsync(layer_jobs.ptr, h_lj, sizeof(LayerJob) * na, hipMemcpyHostToDevice, s),
                         "copy layer jobs")))
            return r;
        if (!dens.empty()) {
            // pageable source: the copy is staged before the call returns
            if ((r = hipfail(hipMemcpy(density.ptr, dens.data(), 8 * dens.size(), hipMemcpyHostToDevice),
                             "copy densities")))
                return r;
        }
        launch_layer_tables(s, na, layer_jobs.ptr, (const double*)density.ptr, (uint8_t*)tables.ptr);
        // phase tables: caller tables, then Mie sets grouped by optics key;
        // every group's jobs sit in their own range of the staging and device
        // job arrays, so no group waits for the previous one
        int n_pj = 0;
        {
            const int g0 = n_pj;
            for (const Req* q : adm) {
                if (q->p.phase_kind != PDV_PHASE_TABLE) continue;
                uint8_t* dst = (uint8_t*)tables.ptr + (uint64_t)q->slot * TableLayout::BYTES + TableLayout::PHASE;
                if ((r = hipfail(hipMemcpy(dst, q->phase.data(), 8 * q->phase.size(), hipMemcpyHostToDevice),
                                 "copy phase table")))
                    return r;
                h_pj[n_pj++] = PhaseJob{1, q->p.n_angles, 0.0, 0.0, (uint64_t)q->slot * TableLayout::BYTES,
                                        q->slot, 0};
            }
            if ((r = launch_phase_group(s, g0, n_pj - g0, 0, nullptr, nullptr))) return r;
        }
        std::vector<char> done(na, 0);
        for (int i = 0; i < na; ++i) {
            if (adm[i]->p.phase_kind != PDV_PHASE_MIE || done[i]) continue;
            if ((r = ctx->ensure_mie_basis(adm[i]->p))) {
                err = ctx->err;
                return r;
            }
            const int g0 = n_pj;
            for (int j = i; j < na; ++j) {
                const pdv_params& p = adm[j]->p;
                if (p.phase_kind != PDV_PHASE_MIE || done[j]) continue;
                MieKey k{p.m_re, p.m_im, p.wavelength, p.d_min, p.d_max, p.n_size_nodes, p.n_angles};
                if (!(k == ctx->mie_key)) continue;
                h_pj[n_pj++] = PhaseJob{0, p.n_angles, p.d_median, p.sigma_ln,
                                        (uint64_t)adm[j]->slot * TableLayout::BYTES, adm[j]->slot, 0};
                done[j] = 1;
            }
            if ((r = launch_phase_group(s, g0, n_pj - g0, ctx->mie_nodes, ctx->mie_info.ptr,
                                        (const double*)ctx->mie_basis.ptr)))
                return r;
        }
        for (const Req* q : adm)
            launch_zero_u64(s, (uint64_t*)tallies.ptr + (uint64_t)q->slot * slot_tally_words(E->opts.max_bins),
                            slot_tally_words(E->opts.max_bins));
        return hipfail(hipGetLastError(), "table kernels");
    }
    int launch_phase_group(hipStream_t s, int first, int n, int n_nodes, const void* info, const double* basis) {
        if (n <= 0) return PDV_OK;
        PhaseJob* dj = (PhaseJob*)phase_jobs.ptr + first;
        int r;
        if ((r = hipfail(hipMemcpyAsync(dj, h_pj + first, sizeof(PhaseJob) * n, hipMemcpyHostToDevice, s),
                         "copy phase jobs")))
            return r;
        launch_phase_cdf(s, n, dj, n_nodes, info, basis, (uint8_t*)tables.ptr, (SetDesc*)descs.ptr,
                         h_pj[first].n_angles);
        return PDV_OK;
    }
    int record(hipStream_t s, const TransportShape& shape) {
        hipError_t e;
        if ((e = hipMemcpyAsync(items.ptr, h_items, sizeof(WorkItem) * max_items, hipMemcpyHostToDevice, s)))
            return hipfail(e, "copy items");
        if ((e = hipMemcpyAsync(nitems.ptr, h_nitems, sizeof(int), hipMemcpyHostToDevice, s)))
            return hipfail(e, "copy item count");
        launch_zero_u64(s, (uint64_t*)queue.ptr, 1);
        e = launch_transport_dev(s, E->opts.precision, shape, (const SetDesc*)descs.ptr, (const uint8_t*)tables.ptr,
                                 (uint64_t*)tallies.ptr, (const WorkItem*)items.ptr, (const int*)nitems.ptr,
                                 (uint32_t*)queue.ptr);
        return hipfail(e, "transport launch");
    }
    std::vector<Req*> copied;    // requests whose results the last launch copied back
    int run(const std::vector<WorkItem>& its, const std::vector<Req*>& finishing, int kind) override {
        copied.clear();
        if (its.empty()) return PDV_OK;
        hipStream_t s = ctx->stream;
        copied = finishing;
        std::memcpy(h_items, its.data(), sizeof(WorkItem) * its.size());
        *h_nitems = (int)its.size();
        const int k = E->opts.precision == PDV_FP64 ? 0 : kind_index(kind);
        int r;
        if (E->opts.use_graph) {
            if (!gexec_k[k]) {
                if ((r = hipfail(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture")))
                    return r;
                const int rr = record(s, shape_k[k]);
                hipError_t e = hipStreamEndCapture(s, &graph_k[k]);
                if (rr) return rr;
                if ((r = hipfail(e, "end capture"))) return r;
                if ((r = hipfail(hipGraphInstantiate(&gexec_k[k], graph_k[k], nullptr, nullptr, 0),
                                 "graph instantiate")))
                    return r;
            }
            if ((r = hipfail(hipGraphLaunch(gexec_k[k], s), "graph launch"))) return r;
        } else {
            if ((r = record(s, shape_k[k]))) return r;
        }
        // the result copies of the requests this launch finishes follow it
        // on the stream, so one wait covers both
        if ((r = copy_results(s, finishing))) return r;
        if (!(E->opts.watchdog_ms > 0.0)) return hipfail(hipStreamSynchronize(s), "transport");
        // bounded wait: poll an event behind the launch and its copies
        if ((r = hipfail(hipEventRecord(ctx->ev_b, s), "watchdog event"))) return r;
        const double deadline = now_s() + 1e-3 * E->opts.watchdog_ms;
        for (;;) {
            const hipError_t q = hipEventQuery(ctx->ev_b);
            if (q == hipSuccess) return PDV_OK;
            if (q != hipErrorNotReady) return hipfail(q, "transport");
            if (now_s() > deadline) {
                ctx->poisoned = true;
                err = "watchdog: launch still running after " + std::to_string(E->opts.watchdog_ms) + " ms";
                return PDV_EDEVICE;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    int copy_results(hipStream_t s, const std::vector<Req*>& reqs) {
        const uint64_t words = slot_tally_words(E->opts.max_bins);
        int r;
        for (Req* q : reqs) {
            const uint64_t off = (uint64_t)q->slot * words;
            if ((r = hipfail(hipMemcpyAsync(h_tally + off, (const uint64_t*)tallies.ptr + off,
                                            8 * tally_words(q->p.n_bins, SF_CLASS), hipMemcpyDeviceToHost, s),
                             "copy tallies")))
                return r;
            if ((r = hipfail(hipMemcpyAsync(h_desc + q->slot, (const SetDesc*)descs.ptr + q->slot, sizeof(SetDesc),
                                            hipMemcpyDeviceToHost, s), "copy descriptor")))
                return r;
        }
        return PDV_OK;
    }
    int collect(const std::vector<Req*>& done, std::vector<int>& st) override {
        const uint64_t words = slot_tally_words(E->opts.max_bins);
        int r;
        // requests the launch did not finish (cancelled ones are not
        // collected) come back here; the others were copied after the launch
        std::vector<Req*> late;
        for (Req* q : done)
            if (std::find(copied.begin(), copied.end(), q) == copied.end()) late.push_back(q);
        if (!late.empty()) {
            if ((r = copy_results(ctx->stream, late))) return r;
            if ((r = hipfail(hipStreamSynchronize(ctx->stream), "copy results"))) return r;
        }
        st.assign(done.size(), PDV_OK);
        for (size_t i = 0; i < done.size(); ++i) {
            Req* q = done[i];
            // the slot's tally block has the request's own n_bins layout
            ctx->unpack(q->p, h_desc[q->slot], h_tally + (uint64_t)q->slot * words, *q->out);
        }
        return PDV_OK;
    }
};

// Host executor for scheduler tests: every packet goes to the "undetected"
// sink with unit weight; optional delay per packet; optional failure.
struct HostExecutor : Executor {
    ServeEngine* E;
    std::vector<std::vector<uint64_t>> slots;
    uint64_t iter = 0;
    std::string err;
    explicit HostExecutor(ServeEngine* e) : E(e) {}
    const char* error() const override { return err.c_str(); }
    int init() override {
        slots.assign(E->opts.max_active, std::vector<uint64_t>(slot_tally_words(E->opts.max_bins), 0));
        return PDV_OK;
    }
    int prepare(const std::vector<Req*>& adm) override {
        for (Req* q : adm) std::fill(slots[q->slot].begin(), slots[q->slot].end(), 0);
        return PDV_OK;
    }
    int run(const std::vector<WorkItem>& its, const std::vector<Req*>&, int) override {
        ++iter;
        if (E->opts.host_fail_iteration && iter == (uint64_t)E->opts.host_fail_iteration) {
            err = "injected executor failure";
            return PDV_EDEVICE;
        }
        uint64_t pk = 0;
        for (const WorkItem& w : its) {
            const int nb = E->active_bins(w.set);
            std::vector<uint64_t>& t = slots[w.set];
            t[tw_sinks(nb) + SK_UNDETECTED] += w.count << 32;
            t[tw_counts(nb) + C_PACKETS] += w.count;
            t[tw_counts(nb) + C_EXITS] += w.count;
            pk += w.count;
        }
        if (E->opts.host_ns_per_packet > 0) {
            const double ns = E->opts.host_ns_per_packet * (double)pk;
            // a launch that outlives the watchdog is given up at the deadline
            if (E->opts.watchdog_ms > 0.0 && ns > 1e6 * E->opts.watchdog_ms) {
                std::this_thread::sleep_for(std::chrono::nanoseconds((uint64_t)(1e6 * E->opts.watchdog_ms)));
                err = "watchdog: launch still running after " + std::to_string(E->opts.watchdog_ms) + " ms";
                return PDV_EDEVICE;
            }
            std::this_thread::sleep_for(std::chrono::nanoseconds((uint64_t)ns));
        }
        return PDV_OK;
    }
    int collect(const std::vector<Req*>& done, std::vector<int>& st) override {
        st.assign(done.size(), PDV_OK);
        for (Req* q : done) {
            SetDesc d;
            std::memset(&d, 0, sizeof d);
            d.albedo = q->p.albedo;
            d.g_mean = q->p.hg_g;
            E->ctx->unpack(q->p, d, slots[q->slot].data(), *q->out);
        }
        return PDV_OK;
    }
};

// ---------------------------------------------------------------------------
// scheduler
// ---------------------------------------------------------------------------
uint64_t ServeEngine::footprint(const Req& r) const {
    uint64_t b = TableLayout::BYTES + 8ull * slot_tally_words(opts.max_bins);
    if (r.want_sg) {
        b += 16ull * r.sg.list_capacity * (uint64_t)r.sg.n_frames;          // detected lists
        b += (uint64_t)r.sg.n_frames * (TableLayout::BYTES + 8ull * tally_words(r.p.n_bins, 0));
        b += 8ull * (uint64_t)r.sg.n_samples + 4ull * (uint64_t)r.sg.nfft * 64;
    }
    return b;
}

int ServeEngine::active_bins(int slot) const { return slot_bins[slot]; }

void ServeEngine::loop() {
    for (;;) {
        std::vector<Req*> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            while (!pending.empty()) {
                std::shared_ptr<Req> q = pending.front();
                if (q->cancel) {
                    pending.pop_front();
                    q->status = PDV_ECANCELLED;
                    q->t_done = now_s();
                    ++n_cancelled;
                    cv_done.notify_all();
                    continue;
                }
                const uint64_t fp = footprint(*q);
                if (free_slots.empty() || mem_in_use + fp > opts.mem_budget) {
                    if (!q->waited) {
                        q->waited = true;
                        ++n_admit_waits;
                    }
                    break;
                }
                pending.pop_front();
                q->slot = free_slots.back();
                free_slots.pop_back();
                slot_bins[q->slot] = q->p.n_bins;
                q->footprint = fp;
                mem_in_use += fp;
                q->t_admit = now_s();
                queue_ms.push_back((q->t_admit - q->t_submit) * 1e3);
                active.push_back(q);
                admitted.push_back(q.get());
            }
            if (active.empty()) {
                if (stopping && (pending.empty() || !drain)) {
                    for (auto& q : pending) {
                        q->status = PDV_ECANCELLED;
                        ++n_cancelled;
                    }
                    pending.clear();
                    cv_done.notify_all();
                    return;
                }
                cv_work.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
        }
        const double t0 = now_s();
        int rc = exec->prepare(admitted);
        const double t_prep = now_s();
        std::vector<WorkItem> items;
        constexpr int KIND_NONE = -2;
        int kind = KIND_NONE;
        std::vector<double> cost;     // estimated work of each item
        if (rc == PDV_OK) {
            std::unique_lock<std::mutex> lk(mu);
            uint64_t open = 0;
            for (auto& q : active)
                if (!q->cancel && q->issued < q->p.n_packets) ++open;
            const uint64_t share = open ? std::max<uint64_t>(opts.packets_per_item, opts.packets_per_iteration / open)
                                        : 0;
            // item size of this iteration: enough items to spread a small
            // iteration over the whole device (results do not depend on it)
            uint64_t total = 0;
            for (auto& q : active)
                if (!q->cancel) total += std::min<uint64_t>(q->p.n_packets - q->issued, share);
            const uint64_t target = 8ull * (uint64_t)std::max(1, ctx->n_cu);
            uint64_t ppi = (total + target - 1) / target;
            ppi = std::max<uint64_t>(ppi, (total + opts.max_items - 1) / (uint64_t)opts.max_items);
            ppi = std::min<uint64_t>(std::max<uint64_t>(ppi, 1024), opts.packets_per_item);
            for (auto& q : active) {
                if (q->cancel) continue;
                uint64_t take = std::min<uint64_t>(q->p.n_packets - q->issued, share);
                if (take > 0 && (int)items.size() < opts.max_items) {
                    // the kernel kind all of this launch's sets share
                    const int k = launch_kind_of(&q->p, 1);
                    kind = (kind == KIND_NONE || kind == k) ? k : KIND_GENERIC;
                }
                while (take > 0 && (int)items.size() < opts.max_items) {
                    const uint64_t c = std::min<uint64_t>(take, ppi);
                    items.push_back(WorkItem{(uint32_t)q->slot, 0, q->p.pid_begin + q->issued, c});
                    cost.push_back((double)c * (1.0 + q->p.tau_total));
                    q->issued += c;
                    take -= c;
                }
            }
            // the most expensive items first (a packet's events grow with
            // the optical depth), so that the persistent blocks' last pulls
            // are short ones and no single long item holds the launch open
            std::vector<int> ord(items.size());
            for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
            std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cost[a] > cost[b]; });
            std::vector<WorkItem> sorted(items.size());
            for (size_t i = 0; i < ord.size(); ++i) sorted[i] = items[ord[i]];
            items.swap(sorted);
        }
        std::vector<Req*> finishing;
        if (rc == PDV_OK) {
            std::unique_lock<std::mutex> lk(mu);
            for (auto& q : active)
                if (!q->cancel && q->issued >= q->p.n_packets) finishing.push_back(q.get());
        }
        if (rc == PDV_OK) rc = exec->run(items, finishing, kind == KIND_NONE ? KIND_GENERIC : kind);
        const double t_run = now_s();
        // retire finished requests: one batched copy of their results
        std::vector<std::shared_ptr<Req>> done_now;
        {
            // the statistics are read by pdv_serve_report under the same lock
            std::unique_lock<std::mutex> lk(mu);
            busy_s += t_run - t0;
            prepare_s += t_prep - t0;
            launch_s += t_run - t_prep;
            ++n_iterations;
            for (auto& q : active)
                if (rc != PDV_OK || q->cancel || q->issued >= q->p.n_packets) done_now.push_back(q);
        }
        std::vector<Req*> to_copy;
        for (auto& q : done_now)
            if (rc == PDV_OK && !q->cancel) to_copy.push_back(q.get());
        std::vector<int> cst;
        if (rc == PDV_OK && !to_copy.empty()) rc = exec->collect(to_copy, cst);
        const double t_col = now_s();
        bool handed = false;
        {
            std::unique_lock<std::mutex> lk(mu);
            collect_s += t_col - t_run;
            if (rc != PDV_OK && fail_msg.empty()) fail_msg = exec->error();
            size_t ci = 0;
            for (auto& q : done_now) {
                int st = rc;
                if (st == PDV_OK && q->cancel) st = PDV_ECANCELLED;
                if (st == PDV_OK) st = cst[ci++];
                // the slot is free once the spectrum is out
                free_slots.push_back(q->slot);
                active.erase(std::find(active.begin(), active.end(), q));
                if (st == PDV_OK && q->want_sg) {
                    sg_queue.push_back(q);          // finished by the spectrogram worker
                    handed = true;
                    continue;
                }
                finish(q, st);
            }
            cv_done.notify_all();
        }
        if (handed) cv_sg.notify_one();
        if (rc != PDV_OK) {
            // the device failed: every waiting request fails the same way
            std::unique_lock<std::mutex> lk(mu);
            failed = true;
            for (auto& q : pending) {
                q->status = rc;
                ++n_failed;
            }
            pending.clear();
            cv_done.notify_all();
            return;
        }
    }
}

void ServeEngine::finish(const std::shared_ptr<Req>& q, int st) {
    q->t_done = now_s();
    if (st == PDV_OK || st == PDV_EOVERFLOW) {
        ++n_completed;
        latencies_ms.push_back((q->t_done - q->t_submit) * 1e3);
        n_packets += q->out->counters.packets;
        n_events += q->out->counters.collisions + q->out->counters.surface;
    } else if (st == PDV_ECANCELLED) {
        ++n_cancelled;
    } else {
        ++n_failed;
    }
    q->status = st;
    mem_in_use -= q->footprint;
}

// Spectrogram worker: frames, beat synthesis and STFT of requests whose
// spectrum is done, on the worker's own context and stream.
void ServeEngine::sg_loop(int worker) {
    pdv_ctx* wctx = sg_ctx[worker];
    for (;;) {
        std::shared_ptr<Req> q;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_sg.wait(lk, [&] { return sg_stop || !sg_queue.empty(); });
            if (sg_queue.empty()) return;
            q = sg_queue.front();
            sg_queue.pop_front();
            if (q->cancel || (sg_stop && !drain)) {
                finish(q, PDV_ECANCELLED);
                cv_done.notify_all();
                continue;
            }
        }
        const double t0 = now_s();
        const int st = pdv_spectrogram_internal(wctx, &q->p, &q->sg, q->sg_out);
        std::unique_lock<std::mutex> lk(mu);
        sg_s += now_s() - t0;
        if (st != PDV_OK && st != PDV_EOVERFLOW && fail_msg.empty()) fail_msg = pdv_last_error(wctx);
        finish(q, st);
        cv_done.notify_all();
    }
}

// Stop the scheduler, then let the spectrogram worker finish (drain) or
// cancel what it still holds, and release its context.
void ServeEngine::join_all() {
    if (th.joinable()) th.join();
    {
        std::unique_lock<std::mutex> lk(mu);
        sg_stop = true;
    }
    cv_sg.notify_all();
    for (std::thread& t : sg_th)
        if (t.joinable()) t.join();
    for (pdv_ctx*& c : sg_ctx) {
        pdv_destroy(c);
        c = nullptr;
    }
    sg_ctx.clear();
}

void pdv_ctx::shutdown_serving() {
    if (!serve) return;
    {
        std::unique_lock<std::mutex> lk(serve->mu);
        serve->stopping = true;
        serve->drain = false;
    }
    serve->cv_work.notify_all();
    serve->join_all();
    serve.reset();
}

pdv_ctx::pdv_ctx() = default;
pdv_ctx::~pdv_ctx() = default;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int pdv_serve_start(pdv_ctx* ctx, const pdv_serve_opts* o) {
    if (!ctx) return PDV_EINVAL;
    if (ctx->serve) return ctx->fail(PDV_ESTATE, "serving already started");
    pdv_serve_opts opts{};
    if (o) opts = *o;
    if (opts.executor != PDV_EXEC_HIP && opts.executor != PDV_EXEC_HOST)
        return ctx->fail(PDV_EINVAL, "unknown executor");
    if (opts.executor == PDV_EXEC_HIP) {
        if (!ctx->ready) return ctx->fail(PDV_ESTATE, "the HIP executor needs a device context");
        if (ctx->poisoned) return ctx->fail(PDV_EDEVICE, "context poisoned by an earlier device error");
    }
    if (opts.max_active <= 0) opts.max_active = 256;
    if (opts.max_items <= 0) opts.max_items = 8192;
    if (opts.packets_per_iteration == 0) opts.packets_per_iteration = 1ull << 25;
    if (opts.packets_per_item == 0) opts.packets_per_item = 1ull << 16;
    if (opts.max_layers <= 0) opts.max_layers = 1024;
    if (opts.max_angles <= 0) opts.max_angles = 2048;
    if (opts.max_bins <= 0) opts.max_bins = 1024;
    if (opts.max_active > 4096 || opts.max_items > (1 << 20) || opts.max_layers > MAX_LAYERS ||
        opts.max_angles > MAX_ANGLES || opts.max_angles < 16 || opts.max_bins > MAX_BINS ||
        opts.packets_per_item > (1ull << 31))
        return ctx->fail(PDV_EINVAL, "serving limits out of range");
    if (opts.precision != PDV_FP32 && opts.precision != PDV_FP64) return ctx->fail(PDV_EINVAL, "bad precision");
    if (!(opts.watchdog_ms >= 0.0) || !std::isfinite(opts.watchdog_ms))
        return ctx->fail(PDV_EINVAL, "watchdog_ms must be finite and >= 0");
    if (opts.sg_workers <= 0) opts.sg_workers = 3;
    if (opts.sg_workers > 8) return ctx->fail(PDV_EINVAL, "sg_workers must be in [1, 8]");
    if (opts.mem_budget == 0) opts.mem_budget = ctx->mem_budget ? ctx->mem_budget / 2 : (1ull << 34);
    auto E = std::make_unique<ServeEngine>();
    E->ctx = ctx;
    E->opts = opts;
    E->slot_bins.assign(opts.max_active, 1);
    for (int s = opts.max_active - 1; s >= 0; --s) E->free_slots.push_back(s);
    if (opts.executor == PDV_EXEC_HIP) E->exec = std::make_unique<HipExecutor>(E.get());
    else E->exec = std::make_unique<HostExecutor>(E.get());
    if (int r = E->exec->init()) {
        std::string msg = E->exec->error();
        if (msg.empty()) msg = ctx->err;
        return ctx->fail(r, "serving executor: %s", msg.c_str());
    }
    if (opts.executor == PDV_EXEC_HIP) {
        // each spectrogram worker's own context: buffers, Mie basis and
        // stream, so the workers' requests overlap on the device
        for (int w = 0; w < opts.sg_workers; ++w) {
            pdv_ctx* c = nullptr;
            const int r = pdv_create(&c, ctx->device, opts.mem_budget, nullptr);
            if (r != PDV_OK) {
                std::string msg = c ? pdv_last_error(c) : "pdv_create failed";
                if (c) pdv_destroy(c);
                for (pdv_ctx* o2 : E->sg_ctx) pdv_destroy(o2);
                E->sg_ctx.clear();
                return ctx->fail(r, "serving spectrogram context: %s", msg.c_str());
            }
            E->sg_ctx.push_back(c);
        }
    }
    E->t_start = now_s();
    ServeEngine* raw = E.get();
    ctx->serve = std::move(E);
    raw->th = std::thread([raw] { raw->loop(); });
    for (int w = 0; w < (int)raw->sg_ctx.size(); ++w) raw->sg_th.emplace_back([raw, w] { raw->sg_loop(w); });
    return PDV_OK;
}

extern "C" int pdv_submit(pdv_ctx* ctx, const pdv_request* req, uint64_t* ticket) {
    if (!ctx || !req || !ticket || !req->out) return PDV_EINVAL;
    ServeEngine* E = ctx->serve.get();
    if (!E) return PDV_ESTATE;
    const pdv_params& p = req->params;
    if (validate_params(nullptr, &p) != PDV_OK) return PDV_EINVAL;
    if (!req->out->w_fx || !req->out->w2_fx) return PDV_EINVAL;
    if (p.flags & PDV_FLAG_DEVICE_OUTPUT) return PDV_EINVAL;   // served results are host arrays
    if (p.flags & PDV_FLAG_PEEL) return PDV_EINVAL;            // served launches carry the ordinary tally only
    if (p.precision != E->opts.precision) return PDV_EINVAL;
    if (p.n_layers > E->opts.max_layers || p.n_bins > E->opts.max_bins ||
        (p.phase_kind != PDV_PHASE_HG && p.n_angles > E->opts.max_angles))
        return PDV_EINVAL;
    auto q = std::make_shared<Req>();
    q->p = p;
    if (p.density_kind == PDV_DENSITY_TABLE) {
        q->density.assign(p.density, p.density + p.n_layers);
        q->p.density = q->density.data();
    }
    if (p.phase_kind == PDV_PHASE_TABLE) {
        q->phase.assign(p.phase, p.phase + p.n_angles);
        q->p.phase = q->phase.data();
    }
    if (req->sg) {
        if (!req->sg_out || !req->sg_out->map) return PDV_EINVAL;
        if (E->opts.executor != PDV_EXEC_HIP) return PDV_EINVAL;
        q->want_sg = true;
        q->sg = *req->sg;
        q->sg_out = req->sg_out;
    }
    q->out = req->out;
    if (E->footprint(*q) > E->opts.mem_budget) return PDV_ENOMEM;
    {
        std::unique_lock<std::mutex> lk(E->mu);
        if (E->stopping || E->failed) return E->failed ? PDV_EDEVICE : PDV_ESTATE;
        q->ticket = E->next_ticket++;
        q->t_submit = now_s();
        E->pending.push_back(q);
        E->by_ticket[q->ticket] = q;
        ++E->n_submitted;
        *ticket = q->ticket;
    }
    E->cv_work.notify_all();
    return PDV_OK;
}

extern "C" int pdv_poll(pdv_ctx* ctx, uint64_t ticket, int32_t wait_ms) {
    if (!ctx) return PDV_EINVAL;
    ServeEngine* E = ctx->serve.get();
    if (!E) return PDV_ESTATE;
    std::unique_lock<std::mutex> lk(E->mu);
    auto it = E->by_ticket.find(ticket);
    if (it == E->by_ticket.end()) return PDV_ENOTFOUND;
    std::shared_ptr<Req> q = it->second;
    auto done = [&] { return q->status != PDV_PENDING; };
    if (!done() && wait_ms != 0) {
        if (wait_ms < 0) E->cv_done.wait(lk, done);
        else E->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), done);
    }
    const int st = q->status;
    if (st != PDV_PENDING) E->by_ticket.erase(ticket);
    return st;
}

extern "C" int pdv_cancel(pdv_ctx* ctx, uint64_t ticket) {
    if (!ctx) return PDV_EINVAL;
    ServeEngine* E = ctx->serve.get();
    if (!E) return PDV_ESTATE;
    std::unique_lock<std::mutex> lk(E->mu);
    auto it = E->by_ticket.find(ticket);
    if (it == E->by_ticket.end()) return PDV_ENOTFOUND;
    it->second->cancel = true;
    E->cv_work.notify_all();
    return PDV_OK;
}

extern "C" int pdv_serve_report(pdv_ctx* ctx, pdv_serve_stats* s) {
    if (!ctx || !s) return PDV_EINVAL;
    ServeEngine* E = ctx->serve.get();
    if (!E) return PDV_ESTATE;
    std::unique_lock<std::mutex> lk(E->mu);
    std::memset(s, 0, sizeof *s);
    s->submitted = E->n_submitted;
    s->completed = E->n_completed;
    s->failed = E->n_failed;
    s->cancelled = E->n_cancelled;
    s->iterations = E->n_iterations;
    s->packets = E->n_packets;
    s->events = E->n_events;
    s->admission_waits = E->n_admit_waits;
    s->active = (uint32_t)E->active.size();
    s->pending = (uint32_t)E->pending.size();
    s->mem_in_use = E->mem_in_use;
    s->busy_s = E->busy_s;
    s->wall_s = now_s() - E->t_start;
    s->prepare_s = E->prepare_s;
    s->launch_s = E->launch_s;
    s->collect_s = E->collect_s;
    s->spectrogram_s = E->sg_s;
    // linear-interpolated percentile of a sorted sample
    auto pct = [](const std::vector<double>& l, double q) {
        const double pos = q * (double)(l.size() - 1);
        const size_t i = (size_t)pos;
        const double f = pos - (double)i;
        return i + 1 < l.size() ? l[i] * (1.0 - f) + l[i + 1] * f : l[i];
    };
    std::vector<double> l = E->latencies_ms;
    if (!l.empty()) {
        std::sort(l.begin(), l.end());
        s->p50_ms = pct(l, 0.50);
        s->p99_ms = pct(l, 0.99);
        s->max_ms = l.back();
        double sum = 0;
        for (double v : l) sum += v;
        s->mean_ms = sum / (double)l.size();
    }
    std::vector<double> w = E->queue_ms;
    if (!w.empty()) {
        std::sort(w.begin(), w.end());
        s->queue_p50_ms = pct(w, 0.50);
    }
    return PDV_OK;
}

extern "C" int pdv_serve_stop(pdv_ctx* ctx, int32_t drain) {
    if (!ctx) return PDV_EINVAL;
    ServeEngine* E = ctx->serve.get();
    if (!E) return PDV_ESTATE;
    {
        std::unique_lock<std::mutex> lk(E->mu);
        E->stopping = true;
        E->drain = drain != 0;
    }
    E->cv_work.notify_all();
    E->join_all();
    const bool failed = E->failed;
    std::string msg = E->fail_msg;
    ctx->serve.reset();
    if (failed) return ctx->fail(PDV_EDEVICE, "serving stopped after an executor failure: %s", msg.c_str());
    return PDV_OK;
}
