// Serving loop of the gpeval library (placeholder until the job loop lands).
#include "runtime.h"

using namespace gpe;

extern "C" {

int gp_server_start(gp_ctx* ctx, const gp_server_cfg* cfg)
{
    (void)cfg;
    return set_err((Ctx*)ctx, GP_EINVAL, "server not available in this build");
}
int gp_server_submit(gp_ctx* ctx, const gp_job* job, int64_t* ticket)
{
    (void)job;
    (void)ticket;
    return set_err((Ctx*)ctx, GP_EINVAL, "server not started");
}
int gp_server_poll(gp_ctx* ctx, int64_t ticket, gp_job_result* out, void* root_out)
{
    (void)ticket;
    (void)out;
    (void)root_out;
    return set_err((Ctx*)ctx, GP_EINVAL, "server not started");
}
int gp_server_release(gp_ctx* ctx, int64_t ticket)
{
    (void)ticket;
    return set_err((Ctx*)ctx, GP_EINVAL, "server not started");
}
int gp_server_stop(gp_ctx* ctx)
{
    (void)ctx;
    return GP_OK;
}
}
