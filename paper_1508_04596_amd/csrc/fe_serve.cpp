// Continuous-batching solve server (scheduler, admission, batched launches).
#include "fe_internal.h"

using namespace fe;

struct fe_server {
    int dummy;
};

extern "C" {

int serve_create(size_t, int, fe_server **out)
{
    if (out) *out = nullptr;
    set_error("serve_create: server not built yet");
    return FE_ESTATE;
}

int serve_submit(fe_server *, const fe_grid *, const fe_phys *, const double *, const double *,
                 const fe_solve_opts *, uint64_t *)
{
    set_error("serve_submit: server not built yet");
    return FE_ESTATE;
}

int serve_poll(fe_server *, uint64_t, double *, fe_solve_report *)
{
    set_error("serve_poll: server not built yet");
    return FE_ESTATE;
}

int serve_times(fe_server *, uint64_t, double *, double *, double *)
{
    set_error("serve_times: server not built yet");
    return FE_ESTATE;
}

int serve_destroy(fe_server *) { return FE_OK; }

}  // extern "C"
