// Stage 2 (placeholder until the beat-synthesis and STFT kernels land).
#include "pdv.h"
#include "pdv_ctx.h"

extern "C" int pdv_spectrogram(pdv_ctx* ctx, const pdv_params*, const pdv_sg_params*, pdv_sg_out*) {
    if (!ctx) return PDV_EINVAL;
    return ctx->fail(PDV_ESTATE, "spectrogram not available in this build");
}
extern "C" int pdv_beat_synthesize(pdv_ctx* ctx, int32_t, const uint64_t*, const float*, const double*,
                                   const uint32_t*, double, double, int32_t, float*) {
    if (!ctx) return PDV_EINVAL;
    return ctx->fail(PDV_ESTATE, "beat synthesis not available in this build");
}
extern "C" int pdv_stft(pdv_ctx* ctx, const float*, int32_t, int32_t, int32_t, float*, int32_t*) {
    if (!ctx) return PDV_EINVAL;
    return ctx->fail(PDV_ESTATE, "stft not available in this build");
}
