// dsdna_noalloc.hip -- the allocation-free entry point: the linking number
// and writhe of caller-supplied closed curves, with the segment-pair
// kernel's per-workgroup partial sums in a fixed device array of this file
// instead of memory the library allocates.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dsdna.h"
#include "dsdna_dev.h"

using namespace dsdna;

namespace {

constexpr int NOALLOC_MAX_BLOCKS = DSDNA_NOALLOC_MAX_POINTS / LK_THREADS;
static_assert(DSDNA_NOALLOC_MAX_POINTS % LK_THREADS == 0, "whole workgroups of curve points");

// Partial sums (Lk, Wr) of each workgroup of the segment-pair kernel.  Every
// GPU the library runs on holds its own copy until the process ends; every
// call on a GPU overwrites the partials of its workgroups before reading them,
// so nothing needs clearing between calls.
static __device__ __align__(256) double scratch[2 * NOALLOC_MAX_BLOCKS];

// Device address of `scratch` on each device, resolved on the first call with
// that device current (the host symbol is only a stand-in for it).
constexpr int MAX_DEVICES = 64;
std::mutex g_mutex;
double *g_scratch[MAX_DEVICES] = {};

dsdna_status scratch_on_current_device(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        set_free_error("no current HIP device (or device index >= %d)", MAX_DEVICES);
        return DSDNA_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_free_error("hipGetSymbolAddress of the scratch array on device %d failed: %s", dev,
                           hipGetErrorString(e));
            return DSDNA_EDEVICE;
        }
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return DSDNA_OK;
}

}  // namespace

extern "C" dsdna_status dsdna_linking_curves_noalloc(const double *A, const double *B, const double *C, int64_t n,
                                                     double *out, void *stream)
{
    if (!A || !B || !C || !out) {
        set_free_error("dsdna_linking_curves_noalloc: null curve or output pointer");
        return DSDNA_EINVAL;
    }
    if (n < 3 || n > DSDNA_NOALLOC_MAX_POINTS) {
        set_free_error("dsdna_linking_curves_noalloc: %lld points per curve, outside [3, %d] (the fixed scratch "
                       "holds %d workgroups of %d points)",
                       (long long)n, DSDNA_NOALLOC_MAX_POINTS, NOALLOC_MAX_BLOCKS, LK_THREADS);
        return DSDNA_EINVAL;
    }
    double *partial = nullptr;
    const dsdna_status st = scratch_on_current_device(&partial);
    if (st != DSDNA_OK) return st;
    const hipError_t e = launch_linking_curves(A, B, C, (int)n, partial, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        set_free_error("dsdna_linking_curves_noalloc: launch failed: %s", hipGetErrorString(e));
        return DSDNA_EDEVICE;
    }
    return DSDNA_OK;
}
