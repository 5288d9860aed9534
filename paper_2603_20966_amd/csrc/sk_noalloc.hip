// sketch_gen_matmul without a caller workspace and without any allocation:
// the FP32 strip partials live in a fixed device array of this library
// (SKETCH_NOALLOC_SCRATCH_BYTES, declared in sketch.h), one copy per GPU,
// held until the process ends.
//
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in symbol, not a device address): the first call on each device looks
// up that device's copy with hipGetSymbolAddress, with the device current, and
// keeps the address; every launch takes that address.  The partials are fully
// written by each call before they are read, so nothing is cleared between
// calls.  Calls that overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "../../include/sketch.h"
#include "sk_internal.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[SKETCH_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch[kMaxDevices];
std::mutex g_scratch_lock;

// Device address of the current device's scratch array (looked up once per
// device, with that device current).
int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return SK_EHIP;
    if (dev >= kMaxDevices) return SK_EUNSUPPORTED;
    void* p = g_scratch[dev].load(std::memory_order_acquire);
    if (p == nullptr) {
        std::lock_guard<std::mutex> guard(g_scratch_lock);
        p = g_scratch[dev].load(std::memory_order_relaxed);
        if (p == nullptr) {
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
                return SK_EHIP;
            g_scratch[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return SK_OK;
}

}  // namespace

extern "C" int sketch_gen_matmul_noalloc(const void* A, int a_dtype, int64_t m, int64_t n,
                                         int64_t lda, const float* a_scales, uint64_t seed,
                                         int64_t omega_row0, int64_t omega_col0, int64_t k,
                                         void* Y, int y_dtype, int64_t ldy, int beta,
                                         void* stream) {
    size_t need = 0;
    int st = sk::gen_matmul_validate(A, a_dtype, m, n, lda, a_scales, SK_DIST_NORMAL, omega_row0,
                                     omega_col0, nullptr, 0, k, Y, y_dtype, ldy, beta, &need);
    if (st == SK_OK && need > (size_t)SKETCH_NOALLOC_SCRATCH_BYTES) st = SK_ESCRATCH;
    void* ws = nullptr;
    if (st == SK_OK && need > 0) st = scratch_address(&ws);
    if (st != SK_OK) {
        sk::drop_trace();
        return st;
    }
    return sk::gen_matmul_impl(A, a_dtype, m, n, lda, a_scales, seed, SK_DIST_NORMAL, omega_row0,
                               omega_col0, nullptr, 0, k, Y, y_dtype, ldy, beta, ws,
                               need > 0 ? (size_t)SKETCH_NOALLOC_SCRATCH_BYTES : 0, stream);
}
