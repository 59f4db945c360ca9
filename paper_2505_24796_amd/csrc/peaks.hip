// Peak-rate probes of the device's vector ALU, transcendental unit and FP16
// matrix cores.  The rasteriser's roofline fractions are stated against the
// rates these probes measure (next to the published ones): every lane runs
// `iters` rounds of eight (four for the matrix cores) independent chains, so
// issue rate rather than dependency latency bounds each probe.
#include "common.h"

namespace {

typedef _Float16 half8_p __attribute__((ext_vector_type(8)));
typedef float f32x16_p __attribute__((ext_vector_type(16)));

enum ProbeKind { PROBE_EXP = 0, PROBE_FMA = 1, PROBE_MFMA_F16 = 2 };

// x <- 2^(-x): v_exp_f32 with a free negation modifier; the chains stay in
// (0.5, 1] for any start in [0, 1].
__global__ __launch_bounds__(256) void k_probe_exp(int iters, float seed, float *__restrict__ out) {
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = seed * (float)((threadIdx.x + 8 * j) & 255) * (1.0f / 256.0f);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = __builtin_amdgcn_exp2f(-x[j]);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += x[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// x <- x * a + b (v_fma_f32, 2 flop per lane); contracts towards b/(1-a).
__global__ __launch_bounds__(256) void k_probe_fma(int iters, float seed, float *__restrict__ out) {
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = seed + (float)j;
    const float a = 0.999f, b = 1.0e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = fmaf(x[j], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += x[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Four independent accumulators of v_mfma_f32_32x32x16_f16 (32768 flop per
// wave instruction), the form the rasteriser's exponent product uses.
__global__ __launch_bounds__(256) void k_probe_mfma(int iters, float seed, float *__restrict__ out) {
    half8_p a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = (_Float16)(seed * 1e-3f * (float)(j + 1));
        b[j] = (_Float16)(1e-3f * (float)((threadIdx.x + j) & 7));
    }
    f32x16_p c0 = {}, c1 = {}, c2 = {}, c3 = {};
    for (int i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c3, 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) s += c0[j] + c1[j] + c2[j] + c3[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" gs_status gs_peak_probe(int32_t kind, int32_t iters, int32_t blocks, float *d_out,
                                   void *stream) {
    if (iters < 1 || blocks < 1 || blocks > (1 << 20) || !d_out || !gs::aligned(d_out, 4))
        return GS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    switch (kind) {
    case PROBE_EXP: hipLaunchKernelGGL(k_probe_exp, dim3(blocks), dim3(256), 0, s, iters, 0.5f, d_out); break;
    case PROBE_FMA: hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, s, iters, 0.5f, d_out); break;
    case PROBE_MFMA_F16:
        hipLaunchKernelGGL(k_probe_mfma, dim3(blocks), dim3(256), 0, s, iters, 0.5f, d_out);
        break;
    default: return GS_ERR_INVALID_ARG;
    }
    return gs::launch_status();
}
