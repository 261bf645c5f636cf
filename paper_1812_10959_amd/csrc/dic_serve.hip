// Serving entry points (placeholder until the continuous-batching scheduler lands).
#include "dic_internal.h"
using namespace dic;
extern "C" {
int dic_serve_create(uint64_t, const dic_serve_opts *, dic_server **out) { if (out) *out = nullptr; set_error("serving not available"); return DIC_E_INVAL; }
int dic_serve_submit(dic_server *, dic_db *, double, uint64_t, uint64_t *) { return DIC_E_INVAL; }
int dic_serve_poll(dic_server *, uint64_t, dic_result **) { return DIC_E_INVAL; }
int dic_serve_wait(dic_server *, uint64_t, int64_t, dic_result **) { return DIC_E_INVAL; }
int dic_serve_stats(dic_server *, double *, double *, double *) { return DIC_E_INVAL; }
int dic_serve_destroy(dic_server *) { return DIC_OK; }
}
