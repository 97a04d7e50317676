// Library context (opaque to ABI users): device, stream, device buffers,
// cached Mie basis, tuning, and the serving engine.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "pdv.h"
#include "pdv_internal.h"

struct DevBuf {
    void* ptr = nullptr;
    size_t cap = 0;
};

struct HostPinned {
    void* ptr = nullptr;
    size_t cap = 0;
};

struct MieKey {
    double m_re, m_im, wavelength, d_min, d_max;
    int32_t n_nodes, n_angles;
    bool operator==(const MieKey& o) const {
        return m_re == o.m_re && m_im == o.m_im && wavelength == o.wavelength && d_min == o.d_min &&
               d_max == o.d_max && n_nodes == o.n_nodes && n_angles == o.n_angles;
    }
};

struct TunedLaunch {
    int32_t block_size = 0;
    int32_t blocks_per_cu = 0;
    uint64_t packets_per_item = 0;
    int32_t persistent = -1;
    int32_t guide_bits = 0;
    int32_t retire_batch = 0;
};

// What a captured batch graph was recorded with.
struct BatchGraphKey {
    int precision = -1, list = 0, persistent = 0, grid = 0, block = 0, lds = 0, guide_bits = 0, retire_min = 0;
    int kind = -1, peel = 0;
    int max_layers = 0, max_cells = 0, max_bins = 0;
    void* ptr[8] = {};
    bool operator==(const BatchGraphKey& o) const {
        if (precision != o.precision || list != o.list || persistent != o.persistent || grid != o.grid ||
            block != o.block || lds != o.lds || guide_bits != o.guide_bits || retire_min != o.retire_min ||
            kind != o.kind || peel != o.peel ||
            max_layers != o.max_layers || max_cells != o.max_cells || max_bins != o.max_bins)
            return false;
        for (int i = 0; i < 8; ++i)
            if (ptr[i] != o.ptr[i]) return false;
        return true;
    }
};

struct ServeEngine;   // serving loop (serve.cpp)
namespace pdv {
int validate_params(pdv_ctx* ctx, const pdv_params* p);
void fill_desc(SetDesc& d, const pdv_params& p);
}
using ListEntry_ = pdv::ListEntry;

struct pdv_ctx {
    int device = 0;
    int n_cu = 256;
    int lds_per_block = 65536, lds_per_cu = 65536;   // device LDS limits (bytes)
    std::string arch;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool ready = false;
    bool poisoned = false;
    uint64_t mem_budget = 0, mem_used = 0;
    std::string err;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;

    // batch buffers
    DevBuf descs, tables, tallies, items, queue, layer_jobs, phase_jobs, density, lists, list_counts, dup_src;
    DevBuf n_items_dev;                  // item count read by graph replays
    DevBuf copy_jobs;                    // device-to-device output copies
    DevBuf pk_in, pk_smooth, pk_out;     // peak analysis
    DevBuf ej_out;                       // ejecta front end
    int h_n_items = 0;
    hipGraphExec_t batch_gexec = nullptr;
    BatchGraphKey batch_key;
    uint64_t graph_captures = 0, graph_replays = 0;
    // Mie basis cache
    DevBuf mie_info, mie_a, mie_b, mie_d, mie_basis, mie_gx, mie_gw;
    MieKey mie_key{};
    bool mie_key_valid = false;
    int mie_nodes = 0;
    // stage-2 buffers
    DevBuf sg_entries, sg_offsets, sg_signal, sg_map, sg_frames, sg_partial, sg_tab;
    int stft_nfft = 0;   // nfft the cached STFT tables were built for
    std::vector<HostPinned> host_pinned;

    // host staging
    std::vector<pdv::SetDesc> h_desc;
    std::vector<pdv::CopyJob> h_copy;    // device-output copies of the last batch
    std::vector<pdv::LayerJob> h_layer;
    std::vector<int> h_src;              // first set with the same tables
    std::vector<pdv::PhaseJob> h_phase;
    std::vector<double> h_density;
    std::vector<pdv::WorkItem> h_items;
    HostPinned tally_pinned;             // pinned staging of a batch's tallies (grow-only)

    // last launch (benchmarks)
    float last_kernel_ms = 0.f;
    int32_t last_grid = 0, last_block = 0, last_items = 0, last_guide_bits = 0, last_lds = 0, last_kind = -1;
    TunedLaunch tuned;

    // serving
    std::unique_ptr<ServeEngine> serve;

    pdv_ctx();
    ~pdv_ctx();
    int fail(int code, const char* fmt, ...);
    int hip_check(hipError_t e, const char* what);
    // true if ptr is device (or managed) memory of this context's device
    bool on_device(const void* ptr);
    int ensure(DevBuf& b, size_t bytes, const char* what);
    int ensure_pinned(HostPinned& b, size_t bytes, const char* what);
    int ensure_mie_basis(const pdv_params& p);
    void default_opts(pdv_launch_opts& o, uint64_t total_packets, int n_sets, bool fp64, int kind,
                      bool list, bool peel = false) const;
    // defer: enqueue the result copies and return without waiting;
    // finish_batch then waits and unpacks
    int run_batch(const pdv_params* sets, int n, pdv_spectrum_out* outs, const pdv_launch_opts* opts,
                  uint64_t list_capacity, bool keep_device, bool defer = false);
    int finish_batch(const pdv_params* sets, int n, pdv_spectrum_out* outs);
    uint64_t pending_tally_words = 0;    // tally words of a deferred batch in tally_pinned
    int synthesize(int n_frames, const uint64_t* entry_begin, const uint64_t* n_entries, const ListEntry_* entries,
                   double wavelength, double fs, int n_samples);
    int synthesize_dev(int n_frames, const uint64_t* d_fbeg, const uint64_t* d_fend, const ListEntry_* entries,
                       uint64_t max_entries, double wavelength, double fs, int n_samples);
    HostPinned counts_pinned;            // list counts of a spectrogram
    int stft(const float* d_signal, int n_samples, int nfft, int hop, int* n_windows);
    void unpack(const pdv_params& p, const pdv::SetDesc& d, const uint64_t* t, pdv_spectrum_out& o);
    int launch_batch_graph(const pdv::TransportShape& sh, int precision, bool list, int persistent);
    void release_all();
    void shutdown_serving();
};
