// VALU issue-rate and vector-memory probe for gfx950 (measurement helper of
// bench.py's roofline; not part of the library).
//
// One kernel per instruction kind, each a long loop of 8 independent chains of
// that one instruction (written in inline assembly so that the compiler can
// neither fold nor reorder them), launched with 8 waves per SIMD on every CU.
// Printed per kind: wave-instructions per second and the issue cycles one
// wave64 instruction takes on its SIMD at the measured clock, which
// classifies each kind as a 2-cycle (dual-issued), 4-cycle or 8-cycle
// instruction.  Run it under rocprofv3 --pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU2
// to see which kinds the second VALU pipe takes.
//
// Two vector-memory kernels follow: coalesced 16-byte loads and 12-byte
// gathers shaped like the adjoint projector's window reads (lane l reads three
// floats starting about two rows after lane l - 1), both from an L2-resident
// buffer.  Run under rocprofv3 --pmc TD_TD_BUSY_sum TA_TA_BUSY_sum
// GRBM_GUI_ACTIVE to see the texture units' busy fraction reach 1 when loads
// alone bound a kernel.
//
// Last, HBM streams over arrays far larger than the caches (4 MB of L2 per XCD,
// 256 MB last-level cache), one element per thread in 256-thread blocks as the
// volume stencils run: a plain copy, a float4 copy, and R reads + 1 write per
// element for the read/write mixes of the stencils.  They give the bandwidth a
// streaming kernel reaches in practice, beside the 8 TB/s of the data sheet.
#include <hip/hip_runtime.h>

#include <cstdio>

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                              \
        }                                                                          \
    } while (0)

constexpr int kChains = 8, kUnroll = 16;

template <int KIND>
__global__ void __launch_bounds__(256) probe(float *out, int iters, float a, float b) {
    float f[kChains];
    unsigned u[kChains];
    const unsigned long long mask = 0x5555555555555555ull;
#pragma unroll
    for (int q = 0; q < kChains; ++q) {
        f[q] = threadIdx.x * 1e-3f + q;
        u[q] = threadIdx.x + q;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < kUnroll; ++r) {
#pragma unroll
            for (int q = 0; q < kChains; ++q) {
                if constexpr (KIND == 0) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(f[q]) : "v"(a), "v"(b));
                if constexpr (KIND == 1) asm volatile("v_add_f32 %0, %0, %1" : "+v"(f[q]) : "v"(b));
                if constexpr (KIND == 2) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(f[q]) : "v"(a));
                if constexpr (KIND == 3) asm volatile("v_add_u32 %0, %0, %1" : "+v"(u[q]) : "v"(it));
                if constexpr (KIND == 4) asm volatile("v_and_b32 %0, %0, %1" : "+v"(u[q]) : "v"(it));
                if constexpr (KIND == 5) asm volatile("v_min_f32 %0, %0, %1" : "+v"(f[q]) : "v"(b));
                if constexpr (KIND == 6) asm volatile("v_med3_f32 %0, %0, %1, %2" : "+v"(f[q]) : "v"(a), "v"(b));
                if constexpr (KIND == 7) asm volatile("v_cvt_flr_i32_f32 %0, %1" : "=v"(u[q]) : "v"(f[q]));
                if constexpr (KIND == 8) asm volatile("v_mul_i32_i24 %0, %0, %1" : "+v"(u[q]) : "v"(it));
                if constexpr (KIND == 9) asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(f[q]) : "v"(a), "s"(mask));
                if constexpr (KIND == 10) asm volatile("v_fma_mix_f32 %0, %1, %2, %0 op_sel_hi:[0,1,0]" : "+v"(f[q]) : "v"(a), "v"(u[q]));
                if constexpr (KIND == 11) asm volatile("v_rcp_f32 %0, %0" : "+v"(f[q]));
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < kChains; ++q) s += f[q] + (float)u[q];
    if (s == 12345.678f) out[blockIdx.x] = s;  // keeps the chains live; never true in practice
}

// Vector-memory probe: KIND 0 coalesced float4 loads, KIND 1 window gathers of
// three floats (lane l at row 2l + (l >> 3), the rows of 64 cells' windows), from
// a buffer of `n` floats that stays in L2; `iters` passes of 64 loads per lane.
template <int KIND>
__global__ void __launch_bounds__(256) vmem(const float *__restrict__ buf, int n, int iters,
                                            float *out) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * 4 + (threadIdx.x >> 6));
    float s = 0.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll 8
        for (int r = 0; r < 64; ++r) {
            if constexpr (KIND == 0) {
                const int o = ((wave * 64 + r) * 256 + lane * 4) & (n - 4);  // 16-byte aligned
                const float4 v = *(const float4 *)(buf + o);
                s += v.x + v.y + v.z + v.w;
            } else {
                const int o = ((wave * 97 + r * 131) * 4 + 2 * lane + (lane >> 3)) & (n - 4);
                s += buf[o] + buf[o + 1] + buf[o + 2];
            }
        }
    }
    if (s == 12345.678f) out[blockIdx.x] = s;  // keeps the loads live; never true in practice
}

template <int R>
struct Ptrs {
    const float *p[R];
};

// out[t] = sum of the R inputs at t: R reads and one write per element.
template <int R>
__global__ void __launch_bounds__(256) stream_mix(Ptrs<R> in, float *__restrict__ out,
                                                  long long n) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < R; ++q) s += in.p[q][t];
    out[t] = s;
}

__global__ void __launch_bounds__(256) stream_copy4(const float4 *__restrict__ a,
                                                    float4 *__restrict__ b, long long n4) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t < n4) b[t] = a[t];
}

// `arrs` holds R + 1 arrays of n floats each: R inputs, then the output.
template <int R>
int run_stream(float *const *arrs, long long n) {
    Ptrs<R> in;
    for (int q = 0; q < R; ++q) in.p[q] = arrs[q];
    float *out = arrs[R];
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(stream_mix<R>, dim3(blocks), dim3(256), 0, 0, in, out, n);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    const int reps = 5;
    CHECK(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(stream_mix<R>, dim3(blocks), dim3(256), 0, 0, in, out, n);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    ms /= reps;
    const double bytes = (R + 1) * 4.0 * (double)n;
    std::printf("stream %2d read + 1 write %9.3f ms  %8.1f GB/s  (%lld floats per array)\n", R, ms,
                bytes / (ms * 1e-3) / 1e9, n);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return 0;
}

int run_copy4(float *a, float *b, long long n) {
    const long long n4 = n / 4;
    const unsigned blocks = (unsigned)((n4 + 255) / 256);
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(stream_copy4, dim3(blocks), dim3(256), 0, 0, (const float4 *)a, (float4 *)b, n4);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    const int reps = 5;
    CHECK(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(stream_copy4, dim3(blocks), dim3(256), 0, 0, (const float4 *)a,
                           (float4 *)b, n4);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    ms /= reps;
    std::printf("stream float4 copy        %9.3f ms  %8.1f GB/s  (%lld floats per array)\n", ms,
                8.0 * (double)n / (ms * 1e-3) / 1e9, n);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return 0;
}

template <int KIND>
int run_vmem(const float *buf, int n, float *out, int blocks, int iters) {
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(vmem<KIND>, dim3(blocks), dim3(256), 0, 0, buf, n, iters, out);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL(vmem<KIND>, dim3(blocks), dim3(256), 0, 0, buf, n, iters, out);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    const double instr = blocks * 4.0 * iters * 64;
    const double bytes = instr * 64 * (KIND == 0 ? 16 : 12);
    std::printf("%-20s %9.3f ms  %8.1f G wave-loads/s  %8.1f GB/s of lane data\n",
                KIND == 0 ? "load float4" : "gather 3 floats", ms, instr / (ms * 1e-3) / 1e9,
                bytes / (ms * 1e-3) / 1e9);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return 0;
}

static const char *kNames[] = {"v_fma_f32", "v_add_f32", "v_mul_f32", "v_add_u32",
                               "v_and_b32", "v_min_f32", "v_med3_f32", "v_cvt_flr_i32_f32",
                               "v_mul_i32_i24", "v_cndmask_b32_e64", "v_fma_mix_f32",
                               "v_rcp_f32"};

template <int KIND>
int run(float *out, int blocks, int iters, int clock_khz) {
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(probe<KIND>, dim3(blocks), dim3(256), 0, 0, out, iters, 0.999f, 0.001f);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    const int reps = 3;
    CHECK(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(probe<KIND>, dim3(blocks), dim3(256), 0, 0, out, iters, 0.999f, 0.001f);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    ms /= reps;
    const double instr = blocks * 4.0 * iters * kUnroll * kChains;  // chain instructions
    const double rate = instr / (ms * 1e-3);
    // issue cycles per wave64 instruction per SIMD at the nominal 2.4 GHz (256 CUs x 4 SIMDs)
    const double cycles = 256.0 * 4.0 * 2.4e9 / rate;
    std::printf("%-20s %9.3f ms  %8.1f G wave-instr/s  %5.2f issue cycles (2.4 GHz)\n",
                kNames[KIND], ms, rate / 1e9, cycles);
    (void)clock_khz;
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return 0;
}

int main() {
    const int blocks = 8192;  // 32 waves per CU: 8 per SIMD on 256 CUs
    const int iters = 4000;
    float *out = nullptr;
    CHECK(hipMalloc(&out, sizeof(float) * blocks));
    int clk = 0;
    CHECK(hipDeviceGetAttribute(&clk, hipDeviceAttributeClockRate, 0));
    std::printf("VALU issue-rate probe: %d blocks x 256 threads, %d x %d x %d instructions per "
                "thread and kind\n", blocks, iters, kUnroll, kChains);
    int rc = 0;
    rc |= run<0>(out, blocks, iters, clk);
    rc |= run<1>(out, blocks, iters, clk);
    rc |= run<2>(out, blocks, iters, clk);
    rc |= run<3>(out, blocks, iters, clk);
    rc |= run<4>(out, blocks, iters, clk);
    rc |= run<5>(out, blocks, iters, clk);
    rc |= run<6>(out, blocks, iters, clk);
    rc |= run<7>(out, blocks, iters, clk);
    rc |= run<8>(out, blocks, iters, clk);
    rc |= run<9>(out, blocks, iters, clk);
    rc |= run<10>(out, blocks, iters, clk);
    rc |= run<11>(out, blocks, iters, clk);
    const int n = 1 << 20;  // 4 MB: resident in L2
    float *buf = nullptr;
    CHECK(hipMalloc(&buf, sizeof(float) * n));
    CHECK(hipMemset(buf, 0, sizeof(float) * n));
    rc |= run_vmem<0>(buf, n, out, blocks, 40);
    rc |= run_vmem<1>(buf, n, out, blocks, 40);
    CHECK(hipFree(buf));
    CHECK(hipFree(out));
    // 11 arrays of 2^27 floats (512 MB each, 5.6 GB in all)
    const long long ns = 1ll << 27;
    float *arrs[11];
    for (int q = 0; q < 11; ++q) {
        CHECK(hipMalloc(&arrs[q], sizeof(float) * ns));
        CHECK(hipMemset(arrs[q], 0, sizeof(float) * ns));
    }
    rc |= run_copy4(arrs[0], arrs[1], ns);
    rc |= run_stream<1>(arrs, ns);
    rc |= run_stream<2>(arrs, ns);
    rc |= run_stream<4>(arrs, ns);
    rc |= run_stream<10>(arrs, ns);
    for (int q = 0; q < 11; ++q) CHECK(hipFree(arrs[q]));
    return rc;
}
