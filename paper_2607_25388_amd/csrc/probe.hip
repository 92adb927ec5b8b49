// probe.hip -- kernels with a known instruction mix, for checking how the hardware counters
// (rocprofv3 SQ_INSTS_VALU_*) count the sweep kernels' work and which instructions the
// SIMDs issue together.  Instrumentation of the library, not part of the planner.
//
// Every lane of every wave runs `iters` iterations of exactly one v_add_f32, one
// v_mul_f32, one v_fma_f32 and one v_exp_f32 (written as inline assembly so the compiler
// cannot fold, reorder or unroll them away); the loop control is scalar.  Outside the loop
// each lane does three v_add_f32 (combining the four values) and one store.
#include <hip/hip_runtime.h>

#include "sgtp.h"

namespace {

__global__ void __launch_bounds__(64) k_probe_fp32(float *out, int iters) {
    float a = (float)threadIdx.x, m = 1.0f, f = 0.5f, e = 0.0f;
    const float b = 1.0000001f, c = 0.999999f;
    for (int i = 0; i < iters; ++i) {
        asm volatile("v_add_f32 %0, %0, %1" : "+v"(a) : "v"(b));
        asm volatile("v_mul_f32 %0, %0, %1" : "+v"(m) : "v"(c));
        asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(f) : "v"(b), "v"(c));
        asm volatile("v_exp_f32 %0, %1\n\ts_nop 1" : "=v"(e) : "v"(c));
    }
    out[blockIdx.x * 64 + threadIdx.x] = ((a + m) + f) + e;
}

// Issue-class probe: every lane runs `iters` iterations of eight independent instructions
// of one kind (inline assembly, scalar loop control), then combines its eight values with
// seven v_add_f32 and stores them.  KIND 0: v_fma_f32 with vector operands; 1: v_fma_f32
// with one scalar operand; 2: v_min_f32; 3: v_sin_f32 (a transcendental); 4: v_mul_f32 with
// a literal; 5: v_xor_b32; 6: v_cndmask_b32 on a scalar mask; 7: v_med3_f32; 8:
// v_mad_u64_u32 (products into registers nothing reads).
template <int KIND>
__global__ void __launch_bounds__(256) k_probe_issue(float *out, int iters) {
    float a0 = (float)threadIdx.x * 1e-3f, a1 = a0 + 0.1f, a2 = a0 + 0.2f, a3 = a0 + 0.3f, a4 = a0 + 0.4f,
          a5 = a0 + 0.5f, a6 = a0 + 0.6f, a7 = a0 + 0.7f;
    const float b = 0.999999f, c = 1e-7f;
    const unsigned long long mask = __builtin_amdgcn_ballot_w64((threadIdx.x & 1) != 0);
    unsigned long long cy = 0;  // carry-out of the kind-8 products
    for (int i = 0; i < iters; ++i) {
        if (KIND == 0) {
            asm volatile("v_fma_f32 %0, %0, %8, %9\n v_fma_f32 %1, %1, %8, %9\n v_fma_f32 %2, %2, %8, %9\n"
                         "v_fma_f32 %3, %3, %8, %9\n v_fma_f32 %4, %4, %8, %9\n v_fma_f32 %5, %5, %8, %9\n"
                         "v_fma_f32 %6, %6, %8, %9\n v_fma_f32 %7, %7, %8, %9"
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                         : "v"(b), "v"(c));
        } else if (KIND == 1) {
            asm volatile("v_fma_f32 %0, %0, %8, %9\n v_fma_f32 %1, %1, %8, %9\n v_fma_f32 %2, %2, %8, %9\n"
                         "v_fma_f32 %3, %3, %8, %9\n v_fma_f32 %4, %4, %8, %9\n v_fma_f32 %5, %5, %8, %9\n"
                         "v_fma_f32 %6, %6, %8, %9\n v_fma_f32 %7, %7, %8, %9"
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                         : "s"(b), "v"(c));
        } else if (KIND == 2) {
            asm volatile("v_min_f32 %0, %0, %8\n v_min_f32 %1, %1, %8\n v_min_f32 %2, %2, %8\n"
                         "v_min_f32 %3, %3, %8\n v_min_f32 %4, %4, %8\n v_min_f32 %5, %5, %8\n"
                         "v_min_f32 %6, %6, %8\n v_min_f32 %7, %7, %8"
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                         : "v"(b));
        } else if (KIND == 3) {
            asm volatile("v_sin_f32 %0, %0\n v_sin_f32 %1, %1\n v_sin_f32 %2, %2\n v_sin_f32 %3, %3\n"
                         "v_sin_f32 %4, %4\n v_sin_f32 %5, %5\n v_sin_f32 %6, %6\n v_sin_f32 %7, %7\n s_nop 1"
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7));
        } else if (KIND == 4) {  // v_mul_f32 with a literal constant
            asm volatile("v_mul_f32 %0, 0x3f7fffef, %0\n v_mul_f32 %1, 0x3f7fffef, %1\n v_mul_f32 %2, 0x3f7fffef, %2\n"
                         "v_mul_f32 %3, 0x3f7fffef, %3\n v_mul_f32 %4, 0x3f7fffef, %4\n v_mul_f32 %5, 0x3f7fffef, %5\n"
                         "v_mul_f32 %6, 0x3f7fffef, %6\n v_mul_f32 %7, 0x3f7fffef, %7"
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7));
        } else if (KIND == 5) {  // v_xor_b32 (vector operands)
            asm volatile("v_xor_b32 %0, %0, %8\n v_xor_b32 %1, %1, %8\n v_xor_b32 %2, %2, %8\n"
                         "v_xor_b32 %3, %3, %8\n v_xor_b32 %4, %4, %8\n v_xor_b32 %5, %5, %8\n"
                         "v_xor_b32 %6, %6, %8\n v_xor_b32 %7, %7, %8"
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                         : "v"(c));
        } else if (KIND == 6) {  // v_cndmask_b32 on a scalar mask
            asm volatile("v_cndmask_b32_e64 %0, %0, %1, %8\n v_cndmask_b32_e64 %1, %1, %2, %8\n"
                         "v_cndmask_b32_e64 %2, %2, %3, %8\n v_cndmask_b32_e64 %3, %3, %4, %8\n"
                         "v_cndmask_b32_e64 %4, %4, %5, %8\n v_cndmask_b32_e64 %5, %5, %6, %8\n"
                         "v_cndmask_b32_e64 %6, %6, %7, %8\n v_cndmask_b32_e64 %7, %7, %0, %8"
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                         : "s"(mask));
        } else if (KIND == 7) {  // v_med3_f32 (vector operands)
            asm volatile("v_med3_f32 %0, %0, %8, %9\n v_med3_f32 %1, %1, %8, %9\n v_med3_f32 %2, %2, %8, %9\n"
                         "v_med3_f32 %3, %3, %8, %9\n v_med3_f32 %4, %4, %8, %9\n v_med3_f32 %5, %5, %8, %9\n"
                         "v_med3_f32 %6, %6, %8, %9\n v_med3_f32 %7, %7, %8, %9"
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                         : "v"(c), "v"(b));
        } else {  // v_mad_u64_u32 (vector operands), eight independent products
            asm volatile("v_mad_u64_u32 v[100:101], %4, %0, %5, 0\n v_mad_u64_u32 v[102:103], %4, %1, %5, 0\n"
                         "v_mad_u64_u32 v[104:105], %4, %2, %5, 0\n v_mad_u64_u32 v[106:107], %4, %3, %5, 0\n"
                         "v_mad_u64_u32 v[108:109], %4, %0, %5, 0\n v_mad_u64_u32 v[110:111], %4, %1, %5, 0\n"
                         "v_mad_u64_u32 v[112:113], %4, %2, %5, 0\n v_mad_u64_u32 v[114:115], %4, %3, %5, 0"
                         : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "=&s"(cy)
                         : "v"(c)
                         : "v100", "v101", "v102", "v103", "v104", "v105", "v106", "v107", "v108", "v109",
                           "v110", "v111", "v112", "v113", "v114", "v115");
        }
    }
    if (KIND == 8) a0 += (float)(cy & 1u);
    out[blockIdx.x * 256 + threadIdx.x] = ((((((a0 + a1) + a2) + a3) + a4) + a5) + a6) + a7;
}

}  // namespace

extern "C" int sgtp_counter_probe_fp32(float *out, int n_waves, int iters, void *stream) {
    if (!out || n_waves < 1 || iters < 0) return SGTP_EINVAL;
    hipLaunchKernelGGL(k_probe_fp32, dim3(n_waves), dim3(64), 0, (hipStream_t)stream, out, iters);
    return hipGetLastError() == hipSuccess ? SGTP_OK : SGTP_EDEVICE;
}

extern "C" int sgtp_issue_probe(float *out, int kind, int n_blocks, int iters, void *stream) {
    if (!out || kind < 0 || kind > 8 || n_blocks < 1 || iters < 0) return SGTP_EINVAL;
    const hipStream_t st = (hipStream_t)stream;
    switch (kind) {
    case 0: hipLaunchKernelGGL(k_probe_issue<0>, dim3(n_blocks), dim3(256), 0, st, out, iters); break;
    case 1: hipLaunchKernelGGL(k_probe_issue<1>, dim3(n_blocks), dim3(256), 0, st, out, iters); break;
    case 2: hipLaunchKernelGGL(k_probe_issue<2>, dim3(n_blocks), dim3(256), 0, st, out, iters); break;
    case 3: hipLaunchKernelGGL(k_probe_issue<3>, dim3(n_blocks), dim3(256), 0, st, out, iters); break;
    case 4: hipLaunchKernelGGL(k_probe_issue<4>, dim3(n_blocks), dim3(256), 0, st, out, iters); break;
    case 5: hipLaunchKernelGGL(k_probe_issue<5>, dim3(n_blocks), dim3(256), 0, st, out, iters); break;
    case 6: hipLaunchKernelGGL(k_probe_issue<6>, dim3(n_blocks), dim3(256), 0, st, out, iters); break;
    case 7: hipLaunchKernelGGL(k_probe_issue<7>, dim3(n_blocks), dim3(256), 0, st, out, iters); break;
    default: hipLaunchKernelGGL(k_probe_issue<8>, dim3(n_blocks), dim3(256), 0, st, out, iters); break;
    }
    return hipGetLastError() == hipSuccess ? SGTP_OK : SGTP_EDEVICE;
}
