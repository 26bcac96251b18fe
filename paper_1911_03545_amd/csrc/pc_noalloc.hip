// pc_noalloc.hip -- the fixed device scratch behind count_pairs_r_noalloc.
//
// Every device buffer of a no-allocation call (staged inputs, the gridded
// points, the counting-sort scratch, the work list, the histograms) is carved
// out of one file-scope device array instead of being allocated.  Each GPU on
// which the library runs holds its own copy of the array, at its own address,
// until the process ends.  Host code never passes the array's name to a
// kernel (in host code it only stands in for the symbol): the device address
// is looked up once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pc_common.h"
#include "pc_launch.h"

static __device__ __align__(256) unsigned char scratch[PC_NOALLOC_SCRATCH_BYTES];

namespace pc {

hipError_t noalloc_scratch(int device, void **ptr, size_t *bytes)
{
    static std::mutex mu;
    static void *addr[PC_NOALLOC_MAX_DEVICES] = {};
    *ptr = nullptr;
    *bytes = 0;
    if (device < 0 || device >= PC_NOALLOC_MAX_DEVICES)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        // the address is per device: look it up with that device current
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess)
            return e;
        if (cur != device)
            return hipErrorInvalidDevice;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        addr[device] = p;
    }
    *ptr = addr[device];
    *bytes = PC_NOALLOC_SCRATCH_BYTES;
    return hipSuccess;
}

}  // namespace pc
