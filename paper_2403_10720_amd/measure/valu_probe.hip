// valu_probe.hip -- measurement tool, not part of the engine's interface:
// issue-rate probe of the integer VALU operations a guess step is made of,
// to calibrate the integer roofline on the device at hand.  Built into its
// own library (libvalu_probe.so), loaded only by the benchmark and its test.
//
// Every lane runs eight independent chains of one operation (so issue, not
// latency, bounds the loop), `iters` times eight operations per chain; the
// results are folded into one word per lane so nothing is optimised away.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

template <int OP>
__device__ __forceinline__ void probe_op(uint32_t &a, uint32_t b)
{
    if constexpr (OP == 0) {
        asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a) : "v"(b));
    } else if constexpr (OP == 1) {
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(a) : "v"(b));
    } else if constexpr (OP == 2) {
        asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a) : "v"(b));
    } else if constexpr (OP == 3) {
        uint64_t r, carry;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(r), "=s"(carry) : "v"(a), "v"(b));
        a = (uint32_t)r;
    } else if constexpr (OP == 4) {
        asm volatile("v_bitop3_b32 %0, %0, %1, %1 bitop3:0x96" : "+v"(a) : "v"(b));
    } else {
        asm volatile("v_bcnt_u32_b32 %0, %0, %1" : "+v"(a) : "v"(b));
    }
}

template <int OP>
__global__ void __launch_bounds__(256) valu_probe_kernel(uint32_t iters, uint32_t *sink)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a0 = t, a1 = t + 1u, a2 = t + 2u, a3 = t + 3u, a4 = t + 4u, a5 = t + 5u, a6 = t + 6u,
             a7 = t + 7u;
    const uint32_t b = t * 2654435761u + 1u;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            probe_op<OP>(a0, b);
            probe_op<OP>(a1, b);
            probe_op<OP>(a2, b);
            probe_op<OP>(a3, b);
            probe_op<OP>(a4, b);
            probe_op<OP>(a5, b);
            probe_op<OP>(a6, b);
            probe_op<OP>(a7, b);
        }
    }
    sink[t] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}

}  // namespace

// op: 0 v_xor_b32, 1 v_add_u32, 2 v_mul_hi_u32, 3 v_mad_u64_u32,
// 4 v_bitop3_b32 (three-input xor), 5 v_bcnt_u32_b32.  `blocks` workgroups of
// 256 lanes, each lane iters * 64 operations in eight independent chains,
// one folded word per lane to sink (device, blocks * 256 words).  Returns 0,
// -1 for an unknown op, blocks outside 1..65536, iters < 1 or a NULL sink,
// -3 if the launch fails.
extern "C" int valu_probe_launch(int32_t op, int64_t blocks, int32_t iters, uint32_t *sink,
                                 void *stream)
{
    if (op < 0 || op > 5 || blocks < 1 || blocks > 65536 || iters < 1 || sink == nullptr)
        return -1;
    const dim3 g((uint32_t)blocks), b(256);
    const uint32_t it = (uint32_t)iters;
    hipStream_t st = (hipStream_t)stream;
    switch (op) {
    case 0: hipLaunchKernelGGL(valu_probe_kernel<0>, g, b, 0, st, it, sink); break;
    case 1: hipLaunchKernelGGL(valu_probe_kernel<1>, g, b, 0, st, it, sink); break;
    case 2: hipLaunchKernelGGL(valu_probe_kernel<2>, g, b, 0, st, it, sink); break;
    case 3: hipLaunchKernelGGL(valu_probe_kernel<3>, g, b, 0, st, it, sink); break;
    case 4: hipLaunchKernelGGL(valu_probe_kernel<4>, g, b, 0, st, it, sink); break;
    default: hipLaunchKernelGGL(valu_probe_kernel<5>, g, b, 0, st, it, sink); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
