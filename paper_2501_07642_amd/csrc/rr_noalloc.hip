// Allocation-free variant of rr_balance_keys, for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops).  Its scratch -- the count and the draw
// bitmasks that rr_balance_keys keeps in the handle's workspace -- is a fixed file-scope device
// array instead.  Calls only enqueue work on the caller's stream; they call no hipMalloc,
// hipFree, hipMemset or synchronisation.
#include <mutex>
#include <string>

#include "rr_internal.h"

namespace rr {

// 64 MiB per GPU, held until the process ends: a 256-byte count, then 8 S words of bitmask per
// key (S = ceil(n/256) rounded up to a power of two), so at most 2097144 keys at n <= 256,
// 524286 at n <= 1024 and 131071 at n <= 4096 when M32 is asked for (M64 alone needs no bitmasks).
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// In host code `scratch` is a host-side stand-in, not device memory: the device address of
// each GPU's copy is looked up once per device (with that device current) and only that
// address reaches the kernels.
static rr_status scratch_address(int dev, void** out) {
    static std::mutex mu;
    static void* addr[64] = {};
    std::lock_guard<std::mutex> g(mu);
    if (dev < 0 || dev >= 64) {
        set_error("rr_balance_keys_noalloc: device index beyond 63");
        return RR_E_UNSUPPORTED;
    }
    if (!addr[dev]) {
        void* ptr = nullptr;
        RR_HIP(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) {
            set_error("rr_balance_keys_noalloc: no device address for the scratch array");
            return RR_E_DEVICE;
        }
        addr[dev] = ptr;
    }
    *out = addr[dev];
    return RR_OK;
}

}  // namespace rr

using namespace rr;

extern "C" {

rr_status rr_balance_keys_noalloc(rr_problem* p, uint64_t seed, int exact, const uint64_t* d_keys, uint64_t K,
                                  int precision, float* d_M32, float* d_err, double* d_M64, void* stream) {
    if (!p || (K && !d_keys) || !valid_prec(precision) || (!d_M32) != (!d_err) || K > 0xFFFFFFFFull) {
        set_error("rr_balance_keys_noalloc: invalid argument");
        return RR_E_ARG;
    }
    if (K == 0) return RR_OK;
    Problem& P = p->P;
    if (exact && P.n > RR_MAX_N_EXACT) {
        set_error("rr_balance_keys_noalloc: exact keys need n <= 64");
        return RR_E_RANGE;
    }
    if (d_M32 && precision == RR_PREC_GRAM_BF16 && P.metric == RR_METRIC_MAX_SMD) {
        set_error("rr_balance_keys_noalloc: the Gram form has no per-column sums (RR_METRIC_MAX_SMD)");
        return RR_E_ARG;
    }
    int cur = -1;
    RR_HIP(hipGetDevice(&cur));
    if (cur != P.device) {
        set_error("rr_balance_keys_noalloc: the current device is not the handle's device");
        return RR_E_ARG;
    }
    if (d_M32 && precision == RR_PREC_GRAM_BF16 && !P.op_gram) {
        set_error("rr_balance_keys_noalloc: the Gram operands of this handle are not built (a call of "
                  "rr_balance_keys or rr_draw_balance with RR_PREC_GRAM_BF16 builds them)");
        return RR_E_ARG;
    }
    const size_t words = (size_t)8 * P.S;
    const size_t need = 256 + (d_M32 ? sizeof(uint32_t) * words * K : 0);
    if (need > kNoAllocScratchBytes) {
        set_error("rr_balance_keys_noalloc: " + std::to_string(K) + " keys need " + std::to_string(need) +
                  " bytes of scratch, above the " + std::to_string(kNoAllocScratchBytes) + " bytes available (at most " +
                  std::to_string((kNoAllocScratchBytes - 256) / (sizeof(uint32_t) * words)) + " keys at n = " +
                  std::to_string(P.n) + " when M32 is asked for)");
        return RR_E_UNSUPPORTED;
    }
    // the binomial table of the device exists once any handle was prepared on it (rr_prepare)
    const uint64_t* binom = exact ? binom_table_ready(P.device) : nullptr;
    if (exact && !binom) {
        set_error("rr_balance_keys_noalloc: binomial table missing on this device");
        return RR_E_DEVICE;
    }
    void* sp = nullptr;
    const rr_status ss = scratch_address(P.device, &sp);
    if (ss != RR_OK) return ss;
    return balance_keys_enqueue(P, seed, exact != 0, binom, d_keys, K, precision, d_M32, d_err, d_M64,
                                (uint32_t*)sp, (uint32_t*)((char*)sp + 256), (hipStream_t)stream);
}

}  // extern "C"
