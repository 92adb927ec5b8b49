// probe.hip -- a kernel with a known FP32 instruction mix, for checking how the hardware
// counters (rocprofv3 SQ_INSTS_VALU_*_F32) count the sweep kernels' work.  Instrumentation
// of the library, not part of the planner.
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

}  // namespace

extern "C" int sgtp_counter_probe_fp32(float *out, int n_waves, int iters, void *stream) {
    if (!out || n_waves < 1 || iters < 0) return SGTP_EINVAL;
    hipLaunchKernelGGL(k_probe_fp32, dim3(n_waves), dim3(64), 0, (hipStream_t)stream, out, iters);
    return hipGetLastError() == hipSuccess ? SGTP_OK : SGTP_EDEVICE;
}
