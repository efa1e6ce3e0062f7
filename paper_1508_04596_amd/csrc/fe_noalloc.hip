// J v without any device allocation, for callers that cannot allocate (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  Same kernels and same results as fe_jvp on a problem created
// with the same grid, parameters and mask; the two work buffers fe_jvp keeps in
// its problem handle -- the per-node mask bits and the tile-face partial sums
// -- live in a file-scope device array instead, whose address is looked up
// once per device.
#include <mutex>

#include "fe_internal.h"

// One copy per device, held until the process ends.  Host code never uses
// this name as an address: the per-device pointer from hipGetSymbolAddress is
// what goes to kernels.
static __device__ __align__(256) unsigned char scratch[FE_NOALLOC_SCRATCH_BYTES];

namespace fe {
namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array (looked up on the first call
// on that device, with the device current).
int scratch_ptr(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("fe_jvp_noalloc: device index out of range");
        return FE_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "fe_jvp_noalloc: hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[dev]);
    return FE_OK;
}

int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }

}  // namespace

int64_t noalloc_scratch_bytes(const fe_grid &grid, fe_prec prec)
{
    const Geo g = make_geo(grid, fe_phys{});
    const int64_t word = prec == FE_FP32 ? 4 : 8;
    return round256(n_nodes(g)) + n_tiles(g) * BOXN * NF * word;
}

}  // namespace fe

using namespace fe;

extern "C" {

int64_t fe_jvp_noalloc_scratch_bytes(const fe_grid *grid, fe_prec prec)
{
    if (!grid || grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return -1;
    return noalloc_scratch_bytes(*grid, prec);
}

int fe_jvp_noalloc(const fe_grid *grid, const fe_phys *phys, fe_prec prec, const uint8_t *dof_mask,
                   const void *x, const double *gamma, const double *s_elem, const void *v,
                   void *jv, hipStream_t stream)
{
    if (!grid || !phys || !x || !gamma || !s_elem || !v || !jv) {
        set_error("fe_jvp_noalloc: NULL argument");
        return FE_EINVAL;
    }
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || !(grid->h > 0.0)) {
        set_error("fe_jvp_noalloc: grid sizes must be >= 1 and h > 0");
        return FE_EINVAL;
    }
    if (prec != FE_FP64 && prec != FE_FP32) {
        set_error("fe_jvp_noalloc: unknown precision");
        return FE_EINVAL;
    }
    if (!(phys->Ck > 0.0)) {
        set_error("fe_jvp_noalloc: phys.Ck must be > 0");
        return FE_EINVAL;
    }
    const int64_t need = noalloc_scratch_bytes(*grid, prec);
    if (need > (int64_t)FE_NOALLOC_SCRATCH_BYTES) {
        set_error("fe_jvp_noalloc: grid needs " + std::to_string(need) +
                  " bytes of scratch, more than the " + std::to_string(FE_NOALLOC_SCRATCH_BYTES) +
                  " available (use fe_problem_create + fe_jvp)");
        return FE_EINVAL;
    }
    int dev = 0;
    FE_CHECK_HIP(hipGetDevice(&dev));
    unsigned char *base = nullptr;
    int rc = scratch_ptr(dev, &base);
    if (rc) return rc;
    const Geo g = make_geo(*grid, *phys);
    const int64_t nn = n_nodes(g);
    uint8_t *nmask = base;
    void *slots = base + round256(nn);
    // every node's mask bits and every slot entry the combine pass reads are
    // written in this call before they are read: nothing needs clearing
    FE_CHECK_HIP(launch_node_mask(dof_mask, nmask, nn, stream));  // NULL mask: all bits 0
    if (prec == FE_FP64)
        FE_CHECK_HIP((launch_elem<double, double>(OP_JV, g, (const double *)x, (const double *)v,
                                                  gamma, s_elem, nmask, (double *)jv,
                                                  (double *)slots, stream)));
    else
        FE_CHECK_HIP((launch_elem<float, float>(OP_JV, g, (const float *)x, (const float *)v, gamma,
                                                s_elem, nmask, (float *)jv, (float *)slots,
                                                stream)));
    return FE_OK;
}

}  // extern "C"
