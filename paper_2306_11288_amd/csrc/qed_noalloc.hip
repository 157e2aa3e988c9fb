// Work memory of the allocation-free lepton step (qed_step_leptons_noalloc): one file-scope
// device array, `scratch`, that every GPU the library runs on holds for the life of the
// process.  Host code never passes the array's name to a kernel or a copy: in host code the
// name is a host-side stand-in, not a device address.  Its device address is taken once
// per device with hipGetSymbolAddress (with that device current) and kept; kernels receive
// that address as an argument, like the context-owned buffers of the ordinary step.
#include <mutex>
#include "qed_internal.hpp"

namespace qed {
namespace {

constexpr int64_t NA_TILES = NOALLOC_MAX / BLOCK;
constexpr int64_t al256(int64_t b) { return (b + 255) / 256 * 256; }
// layout: staging slots, tile counts, group totals (smallest group: 4 tiles), offsets,
// bases, scan block totals.  The group totals are accumulated by atomics and must start at
// zero; every other part is written before it is read within a call.
constexpr int64_t NA_OFF_STAGING = 0;
constexpr int64_t NA_OFF_COUNTS = NA_OFF_STAGING + al256(NOALLOC_MAX * (int64_t)STAGING_SLOT);
constexpr int64_t NA_GROUPS = NA_TILES / 4 + 1;
constexpr int64_t NA_OFF_GROUPS = NA_OFF_COUNTS + al256(NA_TILES * 4);
constexpr int64_t NA_OFF_TILEOFF = NA_OFF_GROUPS + al256(NA_GROUPS * 4);
constexpr int64_t NA_OFF_LAUNCH = NA_OFF_TILEOFF + al256((NA_TILES + 1) * 8);
constexpr int64_t NA_OFF_SUMS = NA_OFF_LAUNCH + al256(4 * 8);
constexpr int64_t NA_BYTES = NA_OFF_SUMS + al256(SCAN_MAX_BLOCKS * 8);

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex na_mutex;
void *na_ptr[MAX_DEVICES];   // device address of `scratch` on each device (set once)

__global__ void k_zero_i32(int *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

}  // namespace

// Address of this device's scratch array, taken on the first call for the current device.
hipError_t noalloc_scratch(void **ptr) {
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(na_mutex);
    if (!na_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        na_ptr[dev] = p;
    }
    *ptr = na_ptr[dev];
    return hipSuccess;
}

ScanState noalloc_state(void *base) {
    char *b = (char *)base;
    ScanState ss;
    ss.staging = b + NA_OFF_STAGING;
    ss.tile_counts = (int *)(b + NA_OFF_COUNTS);
    ss.group_tot = (int *)(b + NA_OFF_GROUPS);
    ss.tile_off = (int64_t *)(b + NA_OFF_TILEOFF);
    ss.launch = (int64_t *)(b + NA_OFF_LAUNCH);
    ss.sums = (int64_t *)(b + NA_OFF_SUMS);
    return ss;
}

// The group totals must start at zero.  The scan clears what it reads, but the array keeps
// whatever an earlier (possibly interrupted) call left, so every call clears them first (a
// kernel, not a memset: capturable).
hipError_t noalloc_clear(const ScanState &ss, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_i32, dim3(2), dim3(256), 0, s, ss.group_tot, (int)NA_GROUPS);
    return hipGetLastError();
}

}  // namespace qed
