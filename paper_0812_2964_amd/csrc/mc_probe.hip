// mc_probe.hip -- microbenchmarks of the chip resources that bound the sweep
// kernels (mc_probe in include/mc.h): the 32-bit vector ALU for the
// instruction classes of a Metropolis attempt (simple, 32-bit multiplies,
// 64-bit multiply-add, three-input bit operations), LDS bandwidth and the
// latency of dependent LDS reads, and the issue interval of a lone wave for
// dependent and for independent instructions, and the cycles of the quad
// sweep step alone (with its threshold reads, with them moved, without them).
// The measured figures replace
// assumed peaks in the roofline of the sweep kernels: a Markov chain's
// attempts are strictly serial, so what one wave can issue bounds a chain.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mc.h"
#include "mc_internal.h"

namespace mcgpu {

namespace {

constexpr int kUnroll = 16;   // asm groups per loop iteration
constexpr int kQuadProbeL = 32;  // lattice of the quad-step probe (k_quad_step_probe)
constexpr int kChains = 8;    // independent registers per thread

// One group of kChains independent instructions of a class, on registers
// r0..r7 with operand b.  Every instruction is plain VALU work on VGPRs.
template <int OP>
__device__ __forceinline__ void valu_group(uint32_t (&r)[kChains], uint32_t b) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        if constexpr (OP == 0)
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(r[i]) : "v"(b));
        else if constexpr (OP == 1)
            asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(r[i]) : "v"(b));
        else if constexpr (OP == 2)
            asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(r[i]) : "v"(b));
        else if constexpr (OP == 4)
            asm volatile("v_bitop3_b32 %0, %0, %1, %0 bitop3:0x96" : "+v"(r[i]) : "v"(b));
    }
}

// Chip-wide rate of one instruction class: every thread issues iters *
// kUnroll * kChains independent instructions (OP 3: 64-bit multiply-adds on
// four register pairs, the same count).
template <int OP>
__global__ __launch_bounds__(64) void k_valu_rate(uint32_t *out, int iters, uint32_t b) {
    uint32_t r[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) r[i] = threadIdx.x * 0x9E3779B9u + i;
    if constexpr (OP == 3) {
        uint64_t q[kChains];
#pragma unroll
        for (int i = 0; i < kChains; ++i) q[i] = r[i];
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int i = 0; i < kChains; ++i)
                    asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(q[i]) : "v"(b), "v"(r[i]) : "vcc");
        }
#pragma unroll
        for (int i = 0; i < kChains; ++i) r[i] = (uint32_t)q[i] ^ (uint32_t)(q[i] >> 32);
    } else {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) valu_group<OP>(r, b);
        }
    }
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) x ^= r[i];
    out[blockIdx.x * 64 + threadIdx.x] = x;
}

// LDS bandwidth: every thread reads 16 bytes per load at lane-consecutive
// addresses (no bank conflicts), iters * kUnroll loads.
__global__ __launch_bounds__(256) void k_lds_bw(uint32_t *out, int iters) {
    __shared__ uint4 buf[4096];  // 64 KB
    for (int i = threadIdx.x; i < 4096; i += 256) buf[i] = make_uint4(i, i * 3u, i * 5u, i * 7u);
    __syncthreads();
    uint4 acc = make_uint4(0, 0, 0, 0);
    for (int it = 0; it < iters; ++it) {
        // the same addresses repeat every iteration: without this barrier the
        // compiler would read them once and reuse the values
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint4 v = buf[(threadIdx.x + 256u * (uint32_t)u) & 4095u];
            acc.x ^= v.x;
            acc.y ^= v.y;
            acc.z ^= v.z;
            acc.w ^= v.w;
        }
    }
    out[blockIdx.x * 256 + threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

// Latency of dependent LDS reads: one wave follows a cycle of indices through
// LDS (each read's address is the previous read's value), iters * kUnroll
// reads, timed with the shader clock.
__global__ __launch_bounds__(64) void k_lds_latency(uint32_t *out, int64_t *cycles, int iters) {
    __shared__ uint32_t nxt[4096];
    for (int i = threadIdx.x; i < 4096; i += 64) nxt[i] = (uint32_t)(i + 65) & 4095u;
    __syncthreads();
    uint32_t p = threadIdx.x;
    const int64_t t0 = clock64();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) p = nxt[p];
    }
    const int64_t t1 = clock64();
    out[threadIdx.x] = p;
    if (threadIdx.x == 0) *cycles = t1 - t0;
}

// Issue interval of a lone wave: dependent (each instruction reads the
// previous one's result) or independent (kChains interleaved chains) simple
// VALU instructions (an xor and an add per step, which the compiler cannot
// fold), timed with the shader clock.
template <bool DEP>
__global__ __launch_bounds__(64) void k_issue(uint32_t *out, int64_t *cycles, int iters, uint32_t b) {
    uint32_t r[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) r[i] = threadIdx.x + i;
    const uint32_t c = b * 3u + 1u;
    const int64_t t0 = clock64();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kUnroll / 2; ++u) {
            if constexpr (DEP) {
#pragma unroll
                for (int i = 0; i < kChains; ++i) r[0] = (r[0] ^ b) + c;
            } else {
#pragma unroll
                for (int i = 0; i < kChains; ++i) r[i] = (r[i] ^ b) + c;
            }
        }
    }
    const int64_t t1 = clock64();
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) x ^= r[i];
    out[threadIdx.x] = x;
    if (threadIdx.x == 0) *cycles = t1 - t0;
}

}  // namespace

}  // namespace mcgpu

using namespace mcgpu;

extern "C" mc_status mc_probe(int32_t kind, int32_t iters, void *hip_stream, double *out_host) {
    if (!out_host || kind < 0 || kind > 11 || iters < 1 || iters > (1 << 24)) {
        set_last_error("mc_probe: kind must be 0..11, iters 1..2^24, out_host non-null");
        return MC_EINVAL;
    }
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1) {
        (void)hipGetLastError();
        set_last_error("mc_probe: no HIP device available");
        return MC_ENODEV;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    // chip-wide kinds: 8 one-wave blocks per SIMD (VALU) or two 4-wave blocks
    // per CU (LDS); lone-wave kinds: one block
    const bool chip = kind <= 5;
    const int valu_blocks = n_cu * 4 * 8, lds_blocks = n_cu * 2;
    const size_t n_out = (size_t)(kind == 5 ? lds_blocks * 256 : valu_blocks * 64);
    uint32_t *out = nullptr;
    int64_t *cyc = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    mc_status status = MC_OK;
    if (hipMalloc((void **)&out, n_out * 4) != hipSuccess || hipMalloc((void **)&cyc, 8) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        status = MC_ENOMEM;
    }
    const uint32_t b = 0x9E3779B9u;
    for (int rep = 0; rep < 2 && status == MC_OK; ++rep) {  // the first run warms up
        (void)hipEventRecord(e0, st);
        switch (kind) {
        case 0: hipLaunchKernelGGL(k_valu_rate<0>, dim3(valu_blocks), dim3(64), 0, st, out, iters, b); break;
        case 1: hipLaunchKernelGGL(k_valu_rate<1>, dim3(valu_blocks), dim3(64), 0, st, out, iters, b); break;
        case 2: hipLaunchKernelGGL(k_valu_rate<2>, dim3(valu_blocks), dim3(64), 0, st, out, iters, b); break;
        case 3: hipLaunchKernelGGL(k_valu_rate<3>, dim3(valu_blocks), dim3(64), 0, st, out, iters, b); break;
        case 4: hipLaunchKernelGGL(k_valu_rate<4>, dim3(valu_blocks), dim3(64), 0, st, out, iters, b); break;
        case 5: hipLaunchKernelGGL(k_lds_bw, dim3(lds_blocks), dim3(256), 0, st, out, iters); break;
        case 6: hipLaunchKernelGGL(k_lds_latency, dim3(1), dim3(64), 0, st, out, cyc, iters); break;
        case 7: hipLaunchKernelGGL(k_issue<true>, dim3(1), dim3(64), 0, st, out, cyc, iters, b); break;
        case 8: hipLaunchKernelGGL(k_issue<false>, dim3(1), dim3(64), 0, st, out, cyc, iters, b); break;
        default:
            if (launch_quad_step_probe(kind - 9, iters, cyc, out, st) != hipSuccess) status = MC_EHIP;
            break;
        }
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) status = MC_EHIP;
    }
    float ms = 0.f;
    int64_t cycles = 0;
    if (status == MC_OK && (hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
                            (!chip && hipMemcpy(&cycles, cyc, 8, hipMemcpyDeviceToHost) != hipSuccess)))
        status = MC_EHIP;
    if (status == MC_OK) {
        const double s = ms * 1e-3;
        const double per_thread = (double)iters * kUnroll * (kind <= 4 ? kChains : 1);
        double work;
        if (kind <= 4)
            work = per_thread * valu_blocks * 64;       // lane-instructions
        else if (kind == 5)
            work = per_thread * lds_blocks * 256 * 16;  // bytes
        else if (kind <= 8)
            work = (double)iters * kUnroll * (kind == 6 ? 1 : kChains);  // dependent reads / instructions of the wave
        else
            work = (double)iters * (kQuadProbeL / 4);  // four-site steps of one chain
        out_host[0] = chip ? work / s : (double)cycles / work;  // rate per second, or cycles per item
        out_host[1] = s;
        out_host[2] = work;
        out_host[3] = (double)cycles;
    }
    if (status == MC_ENOMEM) set_last_error("mc_probe: device allocation failed");
    if (status == MC_EHIP) set_last_error("mc_probe: a HIP call failed");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (cyc) (void)hipFree(cyc);
    return status;
}
