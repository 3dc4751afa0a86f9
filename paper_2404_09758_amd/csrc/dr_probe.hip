// dr_probe.hip -- measurement kernel: the throughput of device-scope atomic
// adds in the address patterns that the estimator's scatter produces.
//
// The scatter of Alg. 2 (one AtomicAdd per contributing parameter and
// pixel) is aggregated per tile in LDS here, and each tile then adds its
// per-group sums to the global accumulators with one 64-bit and one 32-bit
// agent-scope atomic per distinct group.  This kernel issues the same kind
// of atomics, with no returned value, in four address patterns, so the
// flush can be judged against the atomic ceiling of the chip.
#include <hip/hip_runtime.h>

#include "dr.h"
#include "dr_device.h"

namespace {

// Element of operation i in a buffer of n elements of `bytes` bytes.
__device__ __forceinline__ unsigned long long probe_elem(unsigned long long i, unsigned long long n, int pattern,
                                                         int bytes) {
    switch (pattern) {
        case DR_PROBE_CONTIGUOUS:       // lane i of a wave: element i (one line per 16 or 32 lanes)
            return i % n;
        case DR_PROBE_LINES: {          // one element per 128-byte line, lines in order
            unsigned long long per = 128ull / (unsigned long long)bytes;
            return (i * per) % n;
        }
        case DR_PROBE_SCATTERED: {      // a hash of i: lanes fall on unrelated lines
            unsigned long long x = i * 0x9E3779B97F4A7C15ull;
            x ^= x >> 29;
            x *= 0xBF58476D1CE4E5B9ull;
            x ^= x >> 32;
            return x % n;
        }
        default:                        // DR_PROBE_CONFLICTING: the 64 lanes of a wave on one element
            return (i >> 6) % n;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_atomic_probe(T* buf, unsigned long long n_elem, unsigned long long n_ops,
                                                      int pattern) {
    unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_ops) return;
    unsigned long long e = probe_elem(i, n_elem, pattern, (int)sizeof(T));
    __hip_atomic_fetch_add(&buf[e], (T)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every float whose bit pattern lies in [lo, hi] (a grid-stride pass):
// the fast sequence against the general one, counting the operands where
// they differ and keeping the least such bit pattern.
__global__ void __launch_bounds__(256) k_math_probe(int op, unsigned lo, unsigned hi,
                                                    unsigned long long* __restrict__ bad,
                                                    unsigned* __restrict__ first) {
    unsigned long long n = (unsigned long long)hi - lo + 1ull;
    unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    unsigned long long cnt = 0;
    unsigned least = 0xFFFFFFFFu;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        unsigned b = lo + (unsigned)i;
        float x = __uint_as_float(b);
        float f, g;
        if (op == DR_PROBE_SQRT) {
            f = sqrt_rn_fast(x);
            g = sqrtf(x);
        } else {
            f = rcp_rn_fast(x);
            g = 1.0f / x;
        }
        if (__float_as_uint(f) != __float_as_uint(g)) {
            ++cnt;
            least = min(least, b);
        }
    }
    if (cnt) {
        atomicAdd(bad, cnt);
        atomicMin(first, least);
    }
}

}  // namespace

extern "C" dr_status dr_probe_math(int32_t op, uint32_t lo, uint32_t hi, uint64_t* bad, uint32_t* first,
                                   void* stream) {
    if (!bad || !first || lo > hi) return DR_E_INVALID;
    if (op != DR_PROBE_SQRT && op != DR_PROBE_RCP) return DR_E_INVALID;
    hipLaunchKernelGGL(k_math_probe, dim3(8192), dim3(256), 0, (hipStream_t)stream, (int)op, lo, hi,
                       (unsigned long long*)bad, first);
    return hipGetLastError() == hipSuccess ? DR_OK : DR_E_HIP;
}

extern "C" dr_status dr_probe_atomics(void* buf, int64_t bytes, int32_t width_bits, int32_t pattern, int64_t n_ops,
                                      void* stream) {
    if (!buf || bytes <= 0 || n_ops <= 0) return DR_E_INVALID;
    if (width_bits != 32 && width_bits != 64) return DR_E_INVALID;
    if (pattern < DR_PROBE_CONTIGUOUS || pattern > DR_PROBE_CONFLICTING) return DR_E_INVALID;
    if (((uintptr_t)buf & 7u) != 0) return DR_E_INVALID;
    const long long elem = width_bits / 8;
    const unsigned long long n_elem = (unsigned long long)(bytes / elem);
    if (n_elem == 0 || n_ops > (1ll << 40)) return DR_E_INVALID;
    const unsigned long long blocks = ((unsigned long long)n_ops + 255ull) / 256ull;
    if (blocks > 0x7fffffffull) return DR_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    if (width_bits == 64)
        hipLaunchKernelGGL(k_atomic_probe<unsigned long long>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (unsigned long long*)buf, n_elem, (unsigned long long)n_ops, (int)pattern);
    else
        hipLaunchKernelGGL(k_atomic_probe<unsigned>, dim3((unsigned)blocks), dim3(256), 0, st, (unsigned*)buf, n_elem,
                           (unsigned long long)n_ops, (int)pattern);
    return hipGetLastError() == hipSuccess ? DR_OK : DR_E_HIP;
}
