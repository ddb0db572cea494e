// Serving entry points (continuous batching).
#include "qmc_internal.h"

void qmc_serve_shutdown(qmc_ctx *ctx) { (void)ctx; }

extern "C" int qmc_submit(qmc_ctx *ctx, const qmc_plan *plan, const qmc_request *req,
                          uint64_t *ticket)
{
    (void)ctx; (void)plan; (void)req; (void)ticket;
    return QMC_EUNSUPPORTED;
}

extern "C" int qmc_poll(qmc_ctx *ctx, uint64_t ticket, qmc_result *out)
{
    (void)ctx; (void)ticket; (void)out;
    return QMC_EUNSUPPORTED;
}

extern "C" int qmc_wait(qmc_ctx *ctx, uint64_t ticket, double timeout_s, qmc_result *out)
{
    (void)ctx; (void)ticket; (void)timeout_s; (void)out;
    return QMC_EUNSUPPORTED;
}

extern "C" int qmc_cancel(qmc_ctx *ctx, uint64_t ticket)
{
    (void)ctx; (void)ticket;
    return QMC_EUNSUPPORTED;
}
