// Objective and gradient for callers that cannot allocate device memory: the scratch space that
// tlrmdd_grad takes from a caller workspace lives here in a fixed array of the library's device
// code instead (one copy per GPU, held until the process ends).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "tlrmdd.h"

namespace {

constexpr size_t SCRATCH_BYTES = size_t(TLRMDD_NOALLOC_SCRATCH_MIB) << 20;

// Device scratch of tlrmdd_grad_noalloc. Host code never passes this name to a kernel or a copy:
// on the host it only stands for the symbol; the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
std::vector<void *> g_scratch;   // device address of `scratch`, per device (set at the first call there)

int scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return tlr::set_error(TLRMDD_HIP_ERROR, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return tlr::set_error(TLRMDD_HIP_ERROR, std::string("hipGetSymbolAddress(scratch): ") +
                                                        hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return TLRMDD_OK;
}

}  // namespace

extern "C" int tlrmdd_grad_noalloc(tlrmdd_plan plan, const void *D, const void *U, const void *theta, double *f_dev,
                                   void *grad_out, int precision, hipStream_t stream) {
    size_t need = 0;
    int st = tlrmdd_workspace_bytes(plan, TLRMDD_OP_GRAD, nullptr, &need);
    if (st != TLRMDD_OK) return st;
    if (need > SCRATCH_BYTES)
        return tlr::set_error(TLRMDD_WORKSPACE, "tlrmdd_grad_noalloc: the plan needs " + std::to_string(need) +
                                                    " bytes of scratch, more than the " +
                                                    std::to_string(SCRATCH_BYTES) + " the library holds");
    void *ws = nullptr;
    if ((st = scratch_address(&ws)) != TLRMDD_OK) return st;
    return tlrmdd_grad(plan, D, U, theta, f_dev, grad_out, precision, ws, SCRATCH_BYTES, stream);
}
