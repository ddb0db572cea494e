// qmc_integrate_noalloc: qmc_integrate for callers that cannot allocate
// device memory.  Every device buffer of the call (lattices, contracted
// coefficients, shifts, the work list, per-item partial sums, group sums
// and violation counters) is carved out of one file-scope device array,
// `scratch`, that the code object reserves on every device the library is
// loaded on.  The kernels, the work list and the summation order are those
// of qmc_integrate, so both entry points give identical bits.
//
// Host code may not pass the array's name to a kernel (that is a host-side
// stand-in, not a device address): its address on each device is looked up
// once with hipGetSymbolAddress while qmc_create makes that device current,
// and only that address is used afterwards.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/qmc.h"
#include "qmc_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[QMC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices] = {};     // address of `scratch` on each device
std::mutex g_setup_mu;
std::mutex g_use_mu[kMaxDevices];      // one call at a time per device

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

} // namespace

// Called by qmc_create with `device` current.
int qmc_noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return QMC_EDEVICE;
    std::lock_guard<std::mutex> g(g_setup_mu);
    if (g_scratch[device]) return QMC_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
        return QMC_EDEVICE;
    g_scratch[device] = ptr;
    return QMC_OK;
}

extern "C" int qmc_integrate_noalloc(qmc_ctx *ctx, const qmc_plan *plan, const double *kin,
                                     int32_t n_points, const qmc_lattice *lat,
                                     const qmc_lattice *lat_per_sector, const double *shifts,
                                     int32_t m, qmc_result *out)
{
    if (!ctx) return QMC_EINVAL;
    if (!out || !out->coeff) return qmc_set_error(ctx, QMC_EINVAL, "null result");
    const int dev = ctx->device;
    if (dev < 0 || dev >= kMaxDevices || !g_scratch[dev])
        return qmc_set_error(ctx, QMC_EDEVICE, "no scratch address for device %d", dev);
    qmc_job job;
    qmc_job_host H;
    int rc = qmc_job_prepare(ctx, plan, kin, n_points, lat, lat_per_sector, shifts, m, 0, 0,
                             &job, H);
    if (rc) return rc;

    // carve the buffers out of the scratch array, each 256-byte aligned
    const size_t ns = plan->secs.size();
    const size_t kst = (size_t)plan->kstride;
    struct Part {
        void **dst;
        size_t bytes;
        const void *src;
    } parts[] = {
        {(void **)&job.d_lat, sizeof(qmc_lat_dev) * ns, H.lats.data()},
        {(void **)&job.d_coef, sizeof(double) * H.coef.size(), H.coef.data()},
        {(void **)&job.d_dcoef, sizeof(double) * H.dcoef.size(), H.dcoef.data()},
        {(void **)&job.d_lam, sizeof(double) * H.lam.size(), H.lam.data()},
        {(void **)&job.d_shift, sizeof(double) * (size_t)m * QMC_DMAX, shifts},
        {(void **)&job.d_items, sizeof(qmc_item) * H.items.size(), H.items.data()},
        {(void **)&job.d_gbeg, sizeof(int32_t) * H.gbeg.size(), H.gbeg.data()},
        {(void **)&job.d_gend, sizeof(int32_t) * H.gend.size(), H.gend.data()},
        {(void **)&job.d_partial, sizeof(double) * (size_t)job.n_items * kst * 4, nullptr},
        {(void **)&job.d_viol, sizeof(int32_t) * (size_t)job.n_items, nullptr},
        {(void **)&job.d_out, sizeof(double) * (size_t)job.n_groups * kst * 2, nullptr},
        {(void **)&job.d_gviol, sizeof(int32_t) * (size_t)job.n_groups, nullptr},
    };
    size_t need = 0;
    for (const Part &p : parts) need += align256(p.bytes);
    if (need > (size_t)QMC_NOALLOC_SCRATCH_BYTES)
        return qmc_set_error(ctx, QMC_EBUDGET,
                             "qmc_integrate_noalloc needs %zu bytes of scratch, limit %zu "
                             "(fewer points, sectors, shifts or larger tiles)",
                             need, (size_t)QMC_NOALLOC_SCRATCH_BYTES);
    unsigned char *base = (unsigned char *)g_scratch[dev];
    size_t off = 0;
    for (const Part &p : parts) {
        *p.dst = base + off;
        off += align256(p.bytes);
    }
    // group sums and counters come back into host vectors (pageable memory)
    std::vector<double> gsum(job.h_out_n);
    std::vector<int32_t> gviol((size_t)job.n_groups);
    job.h_out = gsum.data();
    job.h_gviol = gviol.data();

    // every buffer above is fully written before it is read (inputs by the
    // uploads, partial sums and counters by every item, group sums by the
    // reduction), so nothing is cleared between calls
    hipError_t e = hipSuccess;
    {
        std::lock_guard<std::mutex> g(g_use_mu[dev]);
        e = hipSetDevice(dev);
        for (const Part &p : parts) {
            if (e != hipSuccess) break;
            if (p.src && p.bytes)
                e = hipMemcpyAsync(*p.dst, p.src, p.bytes, hipMemcpyHostToDevice, ctx->stream);
        }
        if (e == hipSuccess) e = qmc_enqueue(&job, false);
        // the group sums are in host memory, and the scratch array is free
        // for the next call, only once the stream has drained
        const hipError_t es = hipStreamSynchronize(ctx->stream);
        if (e == hipSuccess) e = es;
    }
    job.h_out = nullptr;
    job.h_gviol = nullptr;
    if (e != hipSuccess)
        return qmc_set_error(ctx, QMC_EDEVICE, "qmc_integrate_noalloc: %s", hipGetErrorString(e));
    out->kernel_ms = 0.0;
    return qmc_result_fill(&job, gsum.data(), gviol.data(), out);
}
