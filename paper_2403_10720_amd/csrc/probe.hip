// probe.hip -- issue-rate probe of the integer VALU operations a guess step
// is made of, to calibrate the integer roofline on the device at hand.
//
// Every lane runs eight independent chains of one operation (so issue, not
// latency, bounds the loop), `iters` times eight operations per chain; the
// results are folded into one word per lane so nothing is optimised away.
#include "dvc_core.hpp"
#include "dvc_internal.hpp"

namespace dvc {

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

hipError_t launch_valu_probe(int op, uint32_t blocks, uint32_t iters, uint32_t *sink, hipStream_t st)
{
    switch (op) {
    case 0: hipLaunchKernelGGL(valu_probe_kernel<0>, dim3(blocks), dim3(256), 0, st, iters, sink); break;
    case 1: hipLaunchKernelGGL(valu_probe_kernel<1>, dim3(blocks), dim3(256), 0, st, iters, sink); break;
    case 2: hipLaunchKernelGGL(valu_probe_kernel<2>, dim3(blocks), dim3(256), 0, st, iters, sink); break;
    case 3: hipLaunchKernelGGL(valu_probe_kernel<3>, dim3(blocks), dim3(256), 0, st, iters, sink); break;
    case 4: hipLaunchKernelGGL(valu_probe_kernel<4>, dim3(blocks), dim3(256), 0, st, iters, sink); break;
    default: hipLaunchKernelGGL(valu_probe_kernel<5>, dim3(blocks), dim3(256), 0, st, iters, sink); break;
    }
    return hipGetLastError();
}

}  // namespace dvc
