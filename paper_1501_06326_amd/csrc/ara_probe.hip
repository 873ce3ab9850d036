// ara_probe.hip -- measurement probes behind the roofline figures.
//
//  * k_probe_stream: reads a device buffer once with 16-byte non-temporal
//    loads (the access pattern of the event-id stream), the bandwidth a
//    streaming kernel can reach on this part.
//  * k_probe_valu: long chains of one kind of vector instruction (eight
//    independent chains per lane, so the issue rate and not the latency of
//    one chain is measured), the VALU issue rate per kind.
//  * k_probe_draws: the per-draw arithmetic of secondary uncertainty alone --
//    Philox4x32-10 keyed as the analysis keys it, the draw on the 2^-24 grid
//    and the FP32 Beta quantile of section 3.3 -- with none of the trial
//    walk, lookup, queue or accumulation around it.  Its instruction count
//    per draw is the method's own work per draw.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ara_internal.h"
#include "ara_kernels.h"
#include "ara_math.h"

namespace ara {

__global__ __launch_bounds__(256) void k_probe_stream(const int4 *__restrict__ p, int64_t n16,
                                                      uint32_t *__restrict__ sink) {
    typedef int i32x4 __attribute__((ext_vector_type(4)));
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // four 16-byte loads in flight per lane
    for (; i + 3 * stride < n16; i += 4 * stride) {
        i32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            v[u] = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(p + i + u * stride));
#pragma unroll
        for (int u = 0; u < 4; ++u) acc ^= (uint32_t)(v[u].x ^ v[u].y ^ v[u].z ^ v[u].w);
    }
    for (; i < n16; i += stride) {
        const i32x4 v = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(p + i));
        acc ^= (uint32_t)(v.x ^ v.y ^ v.z ^ v.w);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, d, 64);
    if ((threadIdx.x & 63) == 0) atomicXor(sink, acc);
}

// Eight independent chains of one instruction kind per lane, iters rounds.
template <int KIND>
__global__ __launch_bounds__(256) void k_probe_valu(int32_t iters, float fm, float fc, uint32_t im,
                                                    uint32_t ic, float *__restrict__ out) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    float f[8];
    uint32_t u[8];
    double d[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        f[j] = (float)(tid + j) * 1e-7f;
        u[j] = (uint32_t)(tid * 8 + j);
        d[j] = (double)f[j];
    }
    // four rounds per loop branch, so the loop's scalar bookkeeping stays
    // far below the vector instructions it wraps
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (KIND == ARA_PROBE_FMA_F32) f[j] = fmaf(f[j], fm, fc);
            if (KIND == ARA_PROBE_MUL_F32) f[j] = f[j] * fm;
            if (KIND == ARA_PROBE_XAD_U32) u[j] = (u[j] ^ im) + ic;
            if (KIND == ARA_PROBE_MULHI_U32) u[j] = __umulhi(u[j], im);
            if (KIND == ARA_PROBE_MAD_U64_U32) {
                const uint64_t p = (uint64_t)u[j] * im;
                u[j] = (uint32_t)(p >> 32) ^ (uint32_t)p;
            }
            if (KIND == ARA_PROBE_EXP2_F32) f[j] = __builtin_amdgcn_exp2f(f[j]);
            if (KIND == ARA_PROBE_FMA_F64) d[j] = fma(d[j], (double)fm, (double)fc);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += f[j] + (float)u[j] + (float)d[j];
    out[tid] = s;
}

// n draws of one row (shape a, b; FP32 quantile constants lnb2, na, nb):
// draw j of block-wave w is occurrence k = j % 1024 of trial i = j / 1024,
// keyed (k, i, elt_id, 0) as the analysis keys the independent uniform.
__global__ __launch_bounds__(64) void k_probe_draws(int64_t n, PhiloxKeys keys, uint32_t elt_id,
                                                    float a, float b, float lnb2, int32_t na,
                                                    int32_t nb, const float *__restrict__ tab,
                                                    float *__restrict__ x_out) {
    const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (j >= n) return;
    const uint32_t k = (uint32_t)(j & 1023), i = (uint32_t)(j >> 10);
    const uint32_t ju = u24(philox10_x0(make_uint4(k, i, elt_id, 0u), keys));
    const float z = (float)ju * 5.9604644775390625e-08f;
    const float zc = (float)(16777216u - ju) * 5.9604644775390625e-08f;
    bool ok;
    const float x = beta_quantile32(a, b, lnb2, na, nb, z, zc, tab, &ok);
    x_out[j] = ok ? x : -1.0f;
}

__global__ void k_probe_row_consts(float a, float b, int32_t *out) {
    out[0] = cf_terms((double)a, (double)b);
    out[1] = cf_terms((double)b, (double)a);
}

hipError_t launch_probe_stream(const void *src, int64_t n16, uint32_t *sink, int n_cu,
                               hipStream_t s) {
    // eight 256-thread blocks per CU, each lane keeps four loads in flight
    hipLaunchKernelGGL(k_probe_stream, dim3(n_cu * 8), dim3(256), 0, s, (const int4 *)src, n16,
                       sink);
    return hipGetLastError();
}

template <int K>
static void valu_launch(int blocks, int32_t iters, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_probe_valu<K>, dim3(blocks), dim3(256), 0, s, iters, 1.0000001f,
                       1e-9f, 0x9E3779B9u, 0x7F4A7C15u, out);
}

hipError_t launch_probe_valu(int kind, int blocks, int32_t iters, float *out, hipStream_t s) {
    switch (kind) {
    case ARA_PROBE_FMA_F32: valu_launch<ARA_PROBE_FMA_F32>(blocks, iters, out, s); break;
    case ARA_PROBE_MUL_F32: valu_launch<ARA_PROBE_MUL_F32>(blocks, iters, out, s); break;
    case ARA_PROBE_XAD_U32: valu_launch<ARA_PROBE_XAD_U32>(blocks, iters, out, s); break;
    case ARA_PROBE_MULHI_U32: valu_launch<ARA_PROBE_MULHI_U32>(blocks, iters, out, s); break;
    case ARA_PROBE_MAD_U64_U32: valu_launch<ARA_PROBE_MAD_U64_U32>(blocks, iters, out, s); break;
    case ARA_PROBE_EXP2_F32: valu_launch<ARA_PROBE_EXP2_F32>(blocks, iters, out, s); break;
    case ARA_PROBE_FMA_F64: valu_launch<ARA_PROBE_FMA_F64>(blocks, iters, out, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_probe_row_consts(float a, float b, int32_t *d_out, hipStream_t s) {
    hipLaunchKernelGGL(k_probe_row_consts, dim3(1), dim3(1), 0, s, a, b, d_out);
    return hipGetLastError();
}

hipError_t launch_probe_draws(int64_t n, uint64_t seed, uint32_t elt_id, float a, float b,
                              float lnb2, int32_t na, int32_t nb, const float *tab, float *x,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_draws, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, n,
                       philox_keys(seed), elt_id, a, b, lnb2, na, nb, tab, x);
    return hipGetLastError();
}

}  // namespace ara
