// Serving engine: continuous batching of spectrum requests on one GPU.
#include "pdv_ctx.h"

struct ServeEngine {};

void pdv_ctx::shutdown_serving() { serve.reset(); }

pdv_ctx::pdv_ctx() = default;
pdv_ctx::~pdv_ctx() = default;
