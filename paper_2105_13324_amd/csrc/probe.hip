// Issue-rate probes for the ALU roofline of the transport kernels.
//
// Measurement infrastructure, built into its own library (libmcprobe.so) and
// called only by the benchmark: each kernel keeps every SIMD busy with one
// instruction class in long chains of independent operations (eight chains
// per lane, no memory traffic inside the loop), so its wall time gives the
// sustained issue rate of that class.  The classes are the ones the transport
// is made of: Philox's 32x32->64-bit products (v_mad_u64_u32), 32-bit logic
// (v_xor), FP32 fused multiply-adds, and the hardware transcendentals the
// kernels use (v_log, v_sin, v_cos, v_sqrt, v_rcp), plus one Philox4x32-10
// block per iteration as the mixed case (written as in the transport: each
// three-way xor one v_bitop3_b32).  The result is the number of
// lane-operations of the class per second over the whole device.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int CHAINS = 8;

__global__ __launch_bounds__(256) void k_mad64(uint32_t* out, int iters, uint32_t m) {
    uint32_t a[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) a[c] = threadIdx.x * 977u + (uint32_t)c * 131u + blockIdx.x;
    uint32_t acc = 0;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) {
            const uint64_t p = (uint64_t)a[c] * m;
            a[c] = (uint32_t)(p >> 32) ^ (uint32_t)p;
        }
    }
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc ^= a[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_xor(uint32_t* out, int iters, uint32_t m) {
    uint32_t a[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) a[c] = threadIdx.x * 977u + (uint32_t)c * 131u + blockIdx.x;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) a[c] = (a[c] ^ m) + 0x9E3779B9u;
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc ^= a[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_fma(uint32_t* out, int iters, uint32_t m) {
    float a[CHAINS];
    const float s = 0.999f + 1e-9f * (float)m;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) a[c] = 1.0f + 1e-3f * (float)(threadIdx.x + c);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) a[c] = fmaf(a[c], s, 1e-4f);
    }
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc += a[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = __float_as_uint(acc);
}

// One transcendental per chain step plus one full-rate multiply that keeps
// the argument in range; the multiply's share is removed on the host.
template <int OP>
__global__ __launch_bounds__(256) void k_trans(uint32_t* out, int iters, uint32_t m) {
    float a[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) a[c] = 0.25f + 1e-3f * (float)(threadIdx.x + c + (m & 1u));
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) {
            float r;
            if constexpr (OP == 0) r = __builtin_amdgcn_logf(a[c]);
            else if constexpr (OP == 1) r = __builtin_amdgcn_sinf(a[c]);
            else if constexpr (OP == 2) r = __builtin_amdgcn_sqrtf(a[c]);
            else r = __builtin_amdgcn_rcpf(a[c]);
            a[c] = r * -0.75f;
        }
    }
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc += a[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = __float_as_uint(acc);
}

__global__ __launch_bounds__(256) void k_philox(uint32_t* out, int iters, uint32_t seed) {
    uint32_t c0 = blockIdx.x * blockDim.x + threadIdx.x, c1 = 7u, c2 = 0u, c3 = 0u;
    uint32_t acc = 0;
    for (int i = 0; i < iters; ++i) {
        uint32_t x0 = c0, x1 = c1 ^ acc, x2 = (uint32_t)i + c0 * 3u, x3 = c3 ^ c0, k0 = seed, k1 = 0u;
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            const uint64_t p0 = (uint64_t)x0 * 0xD2511F53u;
            const uint64_t p1 = (uint64_t)x2 * 0xCD9E8D57u;
            const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), x1, k0, 0x96);
            const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), x3, k1, 0x96);
            x1 = (uint32_t)p1;
            x3 = (uint32_t)p0;
            x0 = n0;
            x2 = n2;
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        acc ^= x0 ^ x1 ^ x2 ^ x3;
        c2 += 1u;
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc ^ c2;
}

}  // namespace

extern "C" {

// Run each probe kernel on the current device with `blocks` blocks of 256
// threads and `iters` loop iterations, timed with HIP events on `stream`
// (after one untimed launch).  out_ms[k] receives the kernel time in ms for
// probe k: 0 mad64, 1 xor+add, 2 fma, 3 log, 4 sin, 5 sqrt, 6 rcp, 7 Philox
// block.  scratch: device buffer of blocks * 256 uint32 (written, never
// read back).  Returns 0, or the HIP error code.
int mc_probe_issue(int blocks, int iters, uint32_t* scratch, float* out_ms, void* stream) {
    if (blocks < 1 || iters < 8 || !scratch || !out_ms) return -1;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e[2];
    hipError_t err = hipEventCreate(&e[0]);
    if (err != hipSuccess) return (int)err;
    if ((err = hipEventCreate(&e[1])) != hipSuccess) {
        (void)hipEventDestroy(e[0]);
        return (int)err;
    }
    for (int k = 0; k < 8 && err == hipSuccess; ++k) {
        for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
            if (rep == 1) err = hipEventRecord(e[0], s);
            switch (k) {
                case 0: k_mad64<<<blocks, 256, 0, s>>>(scratch, iters, 0xD2511F53u); break;
                case 1: k_xor<<<blocks, 256, 0, s>>>(scratch, iters, 0xCD9E8D57u); break;
                case 2: k_fma<<<blocks, 256, 0, s>>>(scratch, iters, 3u); break;
                case 3: k_trans<0><<<blocks, 256, 0, s>>>(scratch, iters, 0u); break;
                case 4: k_trans<1><<<blocks, 256, 0, s>>>(scratch, iters, 0u); break;
                case 5: k_trans<2><<<blocks, 256, 0, s>>>(scratch, iters, 0u); break;
                case 6: k_trans<3><<<blocks, 256, 0, s>>>(scratch, iters, 0u); break;
                default: k_philox<<<blocks, 256, 0, s>>>(scratch, iters / 8, 5u); break;
            }
            if (err == hipSuccess) err = hipGetLastError();
            if (rep == 1 && err == hipSuccess) err = hipEventRecord(e[1], s);
        }
        if (err == hipSuccess) err = hipEventSynchronize(e[1]);
        if (err == hipSuccess) err = hipEventElapsedTime(&out_ms[k], e[0], e[1]);
    }
    (void)hipEventDestroy(e[0]);
    (void)hipEventDestroy(e[1]);
    return (int)err;
}

}  // extern "C"
