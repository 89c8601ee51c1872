// Serving engine of libskx (continuous batching over OFDFT requests).
#include "../../include/skx.h"

extern "C" {
int skx_engine_create(skx_engine **out, int, size_t, int) { if (out) *out = nullptr; return SKX_E_INVALID; }
int skx_engine_submit(skx_engine *, const skx_request *, uint64_t *) { return SKX_E_INVALID; }
int skx_engine_step(skx_engine *) { return SKX_E_INVALID; }
int skx_engine_poll(skx_engine *, skx_result *, double **, int, int *) { return SKX_E_INVALID; }
int skx_engine_pending(const skx_engine *) { return 0; }
void skx_engine_destroy(skx_engine *) {}
}
