// Issue-rate probe for the ceilings the kernels are measured against.
//
// Not part of the library: a stand-alone program that times, on every CU of
// the device, (1) single VALU encodings that the integrators issue (16
// independent accumulators per lane, so no instruction waits on another),
// (2) chains of dependent FMAs (1 to 16 independent chains per lane), and
// (3) the FP16 matrix-core shapes with one or more independent accumulators
// per wave, each at 1, 2 and 4 waves per SIMD.  Every kernel only computes
// on registers and stores one float per lane at the end.
//
// Output: one line per case with the wave-level instruction rate per CU (or
// the FLOP rate for the matrix cores), from HIP events around 5 launches.

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kThreads = 256;   // 4 waves: one per SIMD of a CU
constexpr int kCUs = 256;

#define CHECK(x)                                                                  \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));          \
            std::exit(1);                                                         \
        }                                                                         \
    } while (0)

// ---- (1) single VALU encodings -------------------------------------------
enum Op { FMAC_E32, FMA_VOP3, FMA_VOP3_NEG, ADD_E32, SUB_E32, MUL_E32, MUL_E64_NEG, FMAMK, SUB_DPP_WAVE_SHL, NOPS };
const char *kOpName[NOPS] = {"v_fmac_f32_e32", "v_fma_f32 (VOP3)", "v_fma_f32 -a (VOP3)", "v_add_f32_e32",
                             "v_sub_f32_e32", "v_mul_f32_e32", "v_mul_f32_e64 -a", "v_fmamk_f32 (literal)",
                             "v_sub_f32_dpp wave_shl:1"};

template <int OP>
__device__ __forceinline__ void op(float &a, float k1, float k2) {
    if constexpr (OP == FMAC_E32) asm volatile("v_fmac_f32_e32 %0, %1, %2" : "+v"(a) : "v"(k1), "v"(k2));
    else if constexpr (OP == FMA_VOP3) asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(a) : "v"(k1), "v"(k2));
    else if constexpr (OP == FMA_VOP3_NEG) asm volatile("v_fma_f32 %0, -%1, %2, %0" : "+v"(a) : "v"(k1), "v"(k2));
    else if constexpr (OP == ADD_E32) asm volatile("v_add_f32_e32 %0, %1, %0" : "+v"(a) : "v"(k1));
    else if constexpr (OP == SUB_E32) asm volatile("v_sub_f32_e32 %0, %1, %0" : "+v"(a) : "v"(k1));
    else if constexpr (OP == MUL_E32) asm volatile("v_mul_f32_e32 %0, %1, %0" : "+v"(a) : "v"(k1));
    else if constexpr (OP == MUL_E64_NEG) asm volatile("v_mul_f32_e64 %0, -%1, %0" : "+v"(a) : "v"(k1));
    else if constexpr (OP == FMAMK) asm volatile("v_fmamk_f32 %0, %0, 0x3eaaaaab, %1" : "+v"(a) : "v"(k1));
    else asm volatile("v_sub_f32_dpp %0, %0, %1 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                      : "+v"(a) : "v"(k1));
}

template <int OP>
__global__ void __launch_bounds__(kThreads) valu_kernel(float *out, float k1in, float k2in, int iters) {
    float a[16];
    const float k1 = k1in + threadIdx.x * 1e-9f, k2 = k2in - threadIdx.x * 1e-9f;
#pragma unroll
    for (int c = 0; c < 16; ++c) a[c] = threadIdx.x * 1e-3f + c;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int c = 0; c < 16; ++c) op<OP>(a[c], k1, k2);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 16; ++c) s += a[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// ---- (2) dependent FMA chains ---------------------------------------------
template <int NC>
__global__ void __launch_bounds__(kThreads) chain_kernel(float *out, float k1in, float k2in, int iters) {
    float a[NC];
    const float k1 = k1in + threadIdx.x * 1e-9f, k2 = k2in - threadIdx.x * 1e-9f;
#pragma unroll
    for (int c = 0; c < NC; ++c) a[c] = threadIdx.x * 1e-3f + c;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int c = 0; c < NC; ++c) asm volatile("v_fmac_f32_e32 %0, %1, %2" : "+v"(a[c]) : "v"(k1), "v"(k2));
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) s += a[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// ---- (3) matrix cores -------------------------------------------------------
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

template <int SHAPE, int NACC>
__global__ void __launch_bounds__(kThreads) mfma_kernel(float *out, int iters) {
    half8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = (_Float16)(threadIdx.x * 1e-3f + i);
        b[i] = (_Float16)(1e-3f * i);
    }
    float s = 0.f;
    if constexpr (SHAPE == 16) {
        f4 acc[NACC];
#pragma unroll
        for (int c = 0; c < NACC; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < NACC; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < NACC; ++c) s += acc[c][0] + acc[c][3];
    } else {
        f16v acc[NACC];
#pragma unroll
        for (int c = 0; c < NACC; ++c)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[c][e] = 0.f;
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < NACC; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < NACC; ++c) s += acc[c][0] + acc[c][15];
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// ---- timing -------------------------------------------------------------------
template <typename L>
double time_ms(L launch) {
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    launch();
    CHECK(hipEventRecord(e0));
    for (int r = 0; r < 5; ++r) launch();
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    CHECK(hipGetLastError());
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return ms / 5.0;
}

template <int OP>
void valu_case(float *out, int wps) {
    const int blocks = kCUs * wps, iters = 1250;
    const double ms = time_ms([&] {
        hipLaunchKernelGGL(valu_kernel<OP>, dim3(blocks), dim3(kThreads), 0, 0, out, 0.999f, 1e-4f, iters);
    });
    const double winst = (double)blocks * (kThreads / 64) * iters * 8 * 16;
    std::printf("valu  %-26s waves/SIMD %d  %8.3f ms  %6.3f wave-instr/ns/CU\n", kOpName[OP], wps, ms,
                winst / kCUs / (ms * 1e6));
}

template <int NC>
void chain_case(float *out, int wps) {
    const int blocks = kCUs * wps, iters = 20000 / NC;
    const double ms = time_ms([&] {
        hipLaunchKernelGGL(chain_kernel<NC>, dim3(blocks), dim3(kThreads), 0, 0, out, 0.999f, 1e-4f, iters);
    });
    const double winst = (double)blocks * (kThreads / 64) * iters * 8 * NC;
    std::printf("chain %2d independent FMA chains     waves/SIMD %d  %8.3f ms  %6.3f wave-instr/ns/CU\n", NC, wps, ms,
                winst / kCUs / (ms * 1e6));
}

template <int SHAPE, int NACC>
void mfma_case(float *out, int wps) {
    const int blocks = kCUs * wps, iters = 4096 / NACC;
    const double ms = time_ms([&] {
        hipLaunchKernelGGL((mfma_kernel<SHAPE, NACC>), dim3(blocks), dim3(kThreads), 0, 0, out, iters);
    });
    const double flops = (double)blocks * (kThreads / 64) * iters * NACC * (SHAPE == 16 ? 16384.0 : 32768.0);
    std::printf("mfma  %s_f16 %d accumulator(s)  waves/SIMD %d  %8.3f ms  %7.1f TFLOP/s\n",
                SHAPE == 16 ? "16x16x32" : "32x32x16", NACC, wps, ms, flops / (ms * 1e-3) / 1e12);
}

}  // namespace

int main() {
    int dev = 0;
    hipDeviceProp_t prop;
    CHECK(hipGetDevice(&dev));
    CHECK(hipGetDeviceProperties(&prop, dev));
    if (prop.multiProcessorCount != kCUs)
        std::printf("note: the device has %d CUs; rates are per CU of a %d-CU grid\n", prop.multiProcessorCount, kCUs);
    float *out = nullptr;
    CHECK(hipMalloc(&out, sizeof(float) * kCUs * 4 * kThreads));   // largest grid: 4 blocks per CU
    for (int wps : {1, 2, 4}) {
        valu_case<FMAC_E32>(out, wps);
        valu_case<FMA_VOP3>(out, wps);
        valu_case<FMA_VOP3_NEG>(out, wps);
        valu_case<ADD_E32>(out, wps);
        valu_case<SUB_E32>(out, wps);
        valu_case<MUL_E32>(out, wps);
        valu_case<MUL_E64_NEG>(out, wps);
        valu_case<FMAMK>(out, wps);
        valu_case<SUB_DPP_WAVE_SHL>(out, wps);
    }
    for (int wps : {1, 2, 4}) {
        chain_case<1>(out, wps);
        chain_case<2>(out, wps);
        chain_case<4>(out, wps);
        chain_case<16>(out, wps);
    }
    for (int wps : {1, 2, 4}) {
        mfma_case<16, 1>(out, wps);
        mfma_case<16, 2>(out, wps);
        mfma_case<32, 1>(out, wps);
        mfma_case<32, 2>(out, wps);
    }
    CHECK(hipFree(out));
    return 0;
}
