// Race check of the serving scheduler on the host executor: client threads
// submit, poll and cancel requests while another thread reads the
// statistics; built with ThreadSanitizer on the host code by
// test_serve_tsan.py.  Exits non-zero if a finished request reports the
// wrong packet count.
#include <atomic>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "pdv.h"

static pdv_params request(uint64_t n, uint32_t stream) {
    pdv_params p;
    std::memset(&p, 0, sizeof p);
    p.wavelength = 1550e-9;
    p.v_bottom = 1000.0;
    p.v_top = 3000.0;
    p.density_kind = PDV_DENSITY_UNIFORM;
    p.n_layers = 100;
    p.tau_total = 0.1;
    p.phase_kind = PDV_PHASE_HG;
    p.hg_g = 0.7;
    p.albedo = 0.9;
    p.surface_law = PDV_SURFACE_UNIFORM_THETA;
    p.v_surface = 1000.0;
    p.surface_albedo = 0.5;
    p.cone_half_angle = 0.0872664626;
    p.v_lo = 0.0;
    p.v_hi = 4000.0;
    p.n_bins = 64;
    p.max_orders = 50;
    p.weighting = PDV_WEIGHT_IMPLICIT;
    p.precision = PDV_FP32;
    p.n_packets = n;
    p.seed = 1;
    p.stream = stream;
    return p;
}

int main() {
    pdv_ctx* ctx = nullptr;
    if (pdv_create_host(&ctx) != PDV_OK) return 2;
    pdv_serve_opts o;
    std::memset(&o, 0, sizeof o);
    o.executor = PDV_EXEC_HOST;
    o.max_active = 8;
    o.packets_per_iteration = 1u << 14;
    o.packets_per_item = 1u << 12;
    o.max_bins = 64;
    o.host_ns_per_packet = 2.0;
    if (pdv_serve_start(ctx, &o) != PDV_OK) return 3;
    std::atomic<int> bad{0}, done{0}, cancelled{0};
    std::atomic<bool> stop_stats{false};
    std::thread stats([&] {
        pdv_serve_stats s;
        while (!stop_stats.load()) {
            pdv_serve_report(ctx, &s);
            std::this_thread::yield();
        }
    });
    std::vector<std::thread> clients;
    for (int c = 0; c < 6; ++c) {
        clients.emplace_back([&, c] {
            for (int j = 0; j < 25; ++j) {
                const uint64_t n = 500 + 977ull * (uint64_t)((c * 31 + j * 7) % 41);
                std::vector<uint64_t> w(64), w2(64);
                pdv_spectrum_out out;
                std::memset(&out, 0, sizeof out);
                out.w_fx = w.data();
                out.w2_fx = w2.data();
                pdv_request r;
                std::memset(&r, 0, sizeof r);
                r.params = request(n, (uint32_t)(c * 100 + j));
                r.out = &out;
                uint64_t t = 0;
                if (pdv_submit(ctx, &r, &t) != PDV_OK) {
                    ++bad;
                    continue;
                }
                if (j % 9 == 4) pdv_cancel(ctx, t);
                const int st = pdv_poll(ctx, t, -1);
                if (st == PDV_ECANCELLED) {
                    ++cancelled;
                } else if (st != PDV_OK || out.counters.packets != n || out.sinks_fx[PDV_SINK_UNDETECTED] != (n << 32)) {
                    ++bad;
                } else {
                    ++done;
                }
            }
        });
    }
    for (auto& t : clients) t.join();
    stop_stats = true;
    stats.join();
    const int rs = pdv_serve_stop(ctx, 1);
    // a second session whose executor fails at its fifth launch while
    // clients are still submitting: every request ends, none hangs
    o.host_fail_iteration = 5;
    int failed = 0;
    if (pdv_serve_start(ctx, &o) != PDV_OK) return 4;
    std::vector<std::thread> fclients;
    std::atomic<int> fdone{0};
    for (int c = 0; c < 4; ++c) {
        fclients.emplace_back([&, c] {
            for (int j = 0; j < 10; ++j) {
                std::vector<uint64_t> w(64), w2(64);
                pdv_spectrum_out out;
                std::memset(&out, 0, sizeof out);
                out.w_fx = w.data();
                out.w2_fx = w2.data();
                pdv_request r;
                std::memset(&r, 0, sizeof r);
                r.params = request(20000, (uint32_t)(1000 + c * 100 + j));
                r.out = &out;
                uint64_t t = 0;
                if (pdv_submit(ctx, &r, &t) == PDV_OK) pdv_poll(ctx, t, -1);
                ++fdone;
            }
        });
    }
    for (auto& t : fclients) t.join();
    failed = pdv_serve_stop(ctx, 1);
    pdv_destroy(ctx);
    std::printf("done %d cancelled %d bad %d stop %d failed-session %d (%d clients done)\n", done.load(),
                cancelled.load(), bad.load(), rs, failed, fdone.load());
    return (bad.load() == 0 && rs == PDV_OK && done.load() + cancelled.load() == 150 && failed == PDV_EDEVICE &&
            fdone.load() == 40)
               ? 0
               : 1;
}
