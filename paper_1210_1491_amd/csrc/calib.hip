// Issue-rate microbenchmarks for the ALU roofline of the walk kernels.
//
// Each kernel runs eight independent dependency chains per lane of one
// instruction kind (or a fixed pair of kinds), on enough waves to fill every
// SIMD, and the host divides the lane-operations by the elapsed device time.
// The ratio to one full-rate lane-op per lane per cycle (256 CUs x 4 SIMDs x
// 16 lanes x clock) is the cost, in issue slots, that the roofline table
// charges for that instruction kind.  Not part of the method: measurement
// support only, in its own library.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 8;

enum Op {
    OP_FMA_F32 = 0,    // v_fma_f32
    OP_FMA_F64,        // v_fma_f64
    OP_MAD_U64_U32,    // v_mad_u64_u32 (+ one v_xor_b32 folding the halves)
    OP_SQRT_F32,       // v_sqrt_f32 (+ one v_mul_f32)
    OP_SIN_F32,        // v_sin_f32
    OP_RSQ_F64,        // v_rsq_f64
    OP_CVT_F64_F32,    // v_cvt_f64_f32 + v_cvt_f32_f64 (a pair)
    OP_BITOP3,         // v_bitop3_b32
    OP_FMA_F32_SIN,    // v_fma_f32 and v_sin_f32 interleaved (a pair)
    OP_FMA_F64_F32,    // v_fma_f64 and v_fma_f32 interleaved (a pair)
    OP_MIN_F64,        // v_min_f64 and v_max_f64 (a pair)
    OP_COS_F32,        // v_cos_f32
    OP_SQRT_ONLY_F32,  // v_sqrt_f32
    OP_ADD_F64,        // v_add_f64
    OP_MAD_ONLY,       // v_mad_u64_u32 (both halves carried on)
    OP_MULHI_U32,      // v_mul_hi_u32
    OP_COUNT
};

template <int OP>
__global__ __launch_bounds__(256) void k_rate(int iters, uint32_t seed, double *out)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    float f[kChains], g[kChains];
    double d[kChains];
    uint32_t u[kChains], w[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
        u[j] = t * 2654435761u + seed + 97u * j;
        w[j] = u[j] ^ 0x5bd1e995u;
        f[j] = 0.25f + 1e-9f * (float)(u[j] & 1023u);
        g[j] = 0.5f + 1e-9f * (float)(u[j] & 511u);
        d[j] = 0.5 + 1e-12 * (double)(u[j] & 1023u);
    }
    const float a = 0.999f + 1e-9f * (float)(seed & 7u), b = 1e-4f;
    const double ad = 0.999 + 1e-12 * (double)(seed & 7u), bd = 1e-4;
    const uint32_t ka = 0xD2511F53u ^ seed, kb = 0x9E3779B9u + seed;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            if constexpr (OP == OP_FMA_F32) f[j] = fmaf(f[j], a, b);
            if constexpr (OP == OP_FMA_F64) d[j] = fma(d[j], ad, bd);
            if constexpr (OP == OP_MAD_U64_U32) {
                const uint64_t p = (uint64_t)u[j] * ka;
                u[j] = (uint32_t)(p >> 32) ^ (uint32_t)p;
            }
            if constexpr (OP == OP_SQRT_F32) f[j] = __builtin_amdgcn_sqrtf(f[j]) * 1.7f;
            if constexpr (OP == OP_SIN_F32) f[j] = __builtin_amdgcn_sinf(f[j]);
            if constexpr (OP == OP_RSQ_F64) d[j] = __builtin_amdgcn_rsq(d[j]);
            if constexpr (OP == OP_CVT_F64_F32) d[j] = (double)(float)d[j];
            if constexpr (OP == OP_BITOP3) u[j] = __builtin_amdgcn_bitop3_b32(u[j], ka, kb + j, 0x96);
            if constexpr (OP == OP_FMA_F32_SIN) {
                f[j] = fmaf(f[j], a, b);
                g[j] = __builtin_amdgcn_sinf(g[j]);
            }
            if constexpr (OP == OP_FMA_F64_F32) {
                d[j] = fma(d[j], ad, bd);
                f[j] = fmaf(f[j], a, b);
            }
            if constexpr (OP == OP_MIN_F64) d[j] = fmax(fmin(d[j], ad), bd);
            if constexpr (OP == OP_COS_F32) f[j] = __builtin_amdgcn_cosf(f[j]);
            if constexpr (OP == OP_SQRT_ONLY_F32) f[j] = __builtin_amdgcn_sqrtf(f[j]);
            if constexpr (OP == OP_ADD_F64) d[j] = d[j] + bd;
            if constexpr (OP == OP_MAD_ONLY) {
                const uint64_t p = (uint64_t)u[j] * ka + (uint64_t)w[j];
                u[j] = (uint32_t)(p >> 32);
                w[j] = (uint32_t)p;
            }
            if constexpr (OP == OP_MULHI_U32) u[j] = __umulhi(u[j], ka);
        }
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += (double)f[j] + (double)g[j] + d[j] + (double)u[j] + (double)w[j];
    if (s == 12345.678) out[0] = s;  // keeps the chains live; never true in practice
}

template <int OP>
hipError_t run(int blocks, int iters, double *out, float *ms)
{
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rate<OP>, dim3(blocks), dim3(256), 0, nullptr, iters / 8, 1u, out);  // warm-up
    (void)hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(k_rate<OP>, dim3(blocks), dim3(256), 0, nullptr, iters, 2u, out);
    (void)hipEventRecord(e1, nullptr);
    e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e;
}

}  // namespace

extern "C" {

int dtn_calib_count(void) { return OP_COUNT; }

// Chain steps per second of kind `op` (chains x iterations x lanes / time;
// one step is one instruction, or the pair or triple of the kind).  Returns 0
// or a HIP error code.
int dtn_calib_rate(int op, int blocks, int iters, double *lane_ops_per_s, float *ms)
{
    if (op < 0 || op >= OP_COUNT || blocks < 1 || iters < 8 || !lane_ops_per_s || !ms) return -1;
    double *out = nullptr;
    hipError_t e = hipMalloc((void **)&out, sizeof(double));
    if (e != hipSuccess) return (int)e;
    switch (op) {
    case OP_FMA_F32: e = run<OP_FMA_F32>(blocks, iters, out, ms); break;
    case OP_FMA_F64: e = run<OP_FMA_F64>(blocks, iters, out, ms); break;
    case OP_MAD_U64_U32: e = run<OP_MAD_U64_U32>(blocks, iters, out, ms); break;
    case OP_SQRT_F32: e = run<OP_SQRT_F32>(blocks, iters, out, ms); break;
    case OP_SIN_F32: e = run<OP_SIN_F32>(blocks, iters, out, ms); break;
    case OP_RSQ_F64: e = run<OP_RSQ_F64>(blocks, iters, out, ms); break;
    case OP_CVT_F64_F32: e = run<OP_CVT_F64_F32>(blocks, iters, out, ms); break;
    case OP_BITOP3: e = run<OP_BITOP3>(blocks, iters, out, ms); break;
    case OP_FMA_F32_SIN: e = run<OP_FMA_F32_SIN>(blocks, iters, out, ms); break;
    case OP_FMA_F64_F32: e = run<OP_FMA_F64_F32>(blocks, iters, out, ms); break;
    case OP_MIN_F64: e = run<OP_MIN_F64>(blocks, iters, out, ms); break;
    case OP_COS_F32: e = run<OP_COS_F32>(blocks, iters, out, ms); break;
    case OP_SQRT_ONLY_F32: e = run<OP_SQRT_ONLY_F32>(blocks, iters, out, ms); break;
    case OP_ADD_F64: e = run<OP_ADD_F64>(blocks, iters, out, ms); break;
    case OP_MAD_ONLY: e = run<OP_MAD_ONLY>(blocks, iters, out, ms); break;
    default: e = run<OP_MULHI_U32>(blocks, iters, out, ms); break;
    }
    (void)hipFree(out);
    if (e != hipSuccess) return (int)e;
    *lane_ops_per_s = (double)blocks * 256.0 * kChains * (double)iters / (*ms * 1e-3);
    return 0;
}

}  // extern "C"
