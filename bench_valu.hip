// bench_valu.hip -- issue rate of single VALU instruction forms on one MI355X (gfx950).
//
// Measurement behind the ALU peak that bench.py prices kernels against.  For each form, every
// thread runs eight independent dependency chains of that one instruction for ITER iterations;
// 4096 work-groups of 256 threads (16384 waves) keep every SIMD of the 256 CUs busy.  Output:
// one line per form, lane-operations per second (one lane-op = one 32-bit lane of one
// instruction), in units of 1e12.
//
// Build and run: bench.py --valu-rates (hipcc --offload-arch=gfx950 -O3 bench_valu.hip).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

constexpr int kIter = 2048;
constexpr int kThreads = 256;
constexpr int kBlocks = 4096;

template <int F>
__device__ __forceinline__ void step(uint32_t &a, uint64_t &w, float &f, uint32_t b, uint32_t c,
                                     uint32_t s, float fb, float fc)
{
    if constexpr (F == 0) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a) : "v"(b));
    if constexpr (F == 1) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a) : "v"(b));
    if constexpr (F == 2) asm volatile("v_lshrrev_b32 %0, 3, %0" : "+v"(a));
    if constexpr (F == 3) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a) : "s"(s));
    if constexpr (F == 4) asm volatile("v_add_u32_e64 %0, %0, %1" : "+v"(a) : "v"(b));
    if constexpr (F == 5) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a) : "v"(b));
    if constexpr (F == 6) asm volatile("v_mul_u32_u24 %0, %0, %1" : "+v"(a) : "v"(b));
    if constexpr (F == 7) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(w) : "v"(a), "v"(b) : "vcc");
    if constexpr (F == 8) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a) : "v"(b), "v"(c));
    if constexpr (F == 9) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a) : "v"(b), "s"(s));
    if constexpr (F == 10) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
    if constexpr (F == 11) asm volatile("v_lshl_add_u32 %0, %0, 2, %1" : "+v"(a) : "v"(b));
    if constexpr (F == 12) asm volatile("v_perm_b32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
    if constexpr (F == 13) asm volatile("v_bfe_u32 %0, %0, 3, 4" : "+v"(a));
    if constexpr (F == 14) asm volatile("v_sub_co_u32_e32 %0, vcc, %0, %1" : "+v"(a) : "v"(b) : "vcc");
    if constexpr (F == 15) asm volatile("v_addc_co_u32_e32 %0, vcc, %0, %1, vcc" : "+v"(a) : "v"(b) : "vcc");
    if constexpr (F == 16) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(f) : "v"(fb), "v"(fc));
    if constexpr (F == 17) asm volatile("v_add_f32 %0, %0, %1" : "+v"(f) : "v"(fb));
    if constexpr (F == 18) asm volatile("v_cndmask_b32 %0, %0, %1, vcc" : "+v"(a) : "v"(b) : "vcc");
}

template <int F>
__global__ __launch_bounds__(kThreads) void rate_kernel(uint32_t *out, uint32_t seed)
{
    uint32_t a[8];
    uint64_t w[8];
    float f[8];
    const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = t * (2 * i + 1) + seed;
        w[i] = a[i];
        f[i] = (float)(a[i] & 255) * 1e-3f;
    }
    const uint32_t b = t ^ seed, c = t + 3 * seed;
    const float fb = 0.999f, fc = 1e-6f;
    for (int it = 0; it < kIter; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) step<F>(a[i], w[i], f[i], b, c, seed + (uint32_t)i, fb, fc);
    }
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) r ^= a[i] ^ (uint32_t)w[i] ^ (uint32_t)(w[i] >> 32) ^ __float_as_uint(f[i]);
    out[t] = r;
}

static const char *kNames[] = {
    "v_xor_b32 v,v", "v_add_u32 v,v", "v_lshrrev_b32 c,v", "v_xor_b32 s,v", "v_add_u32_e64 v,v",
    "v_mul_hi_u32 v,v", "v_mul_u32_u24 v,v", "v_mad_u64_u32 v,v,v[2] (vcc)",
    "v_bitop3_b32 v,v,v", "v_bitop3_b32 v,v,s", "v_add3_u32 v,v,v", "v_lshl_add_u32 v,c,v",
    "v_perm_b32 v,v,v", "v_bfe_u32 v,c,c", "v_sub_co_u32 v,v (writes vcc)",
    "v_addc_co_u32 v,v,vcc", "v_fma_f32 v,v,v", "v_add_f32 v,v", "v_cndmask_b32 v,v,vcc"};

template <int F>
static double run(uint32_t *out, hipEvent_t e0, hipEvent_t e1)
{
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(rate_kernel<F>, dim3(kBlocks), dim3(kThreads), 0, 0, out, 12345u + rep);
        (void)hipEventRecord(e1, 0);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) best = ms;
    }
    const double ops = (double)kBlocks * kThreads * kIter * 8;
    return ops / (best * 1e-3) / 1e12;
}

template <int F>
static void all(uint32_t *out, hipEvent_t e0, hipEvent_t e1)
{
    if constexpr (F < 19) {
        std::printf("%-34s %8.2f\n", kNames[F], run<F>(out, e0, e1));
        all<F + 1>(out, e0, e1);
    }
}

int main()
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, 0) != hipSuccess) {
        std::fprintf(stderr, "no HIP device\n");
        return 1;
    }
    std::printf("# %s, %d CUs, max clock %d MHz; T lane-ops/s per instruction form\n", p.gcnArchName,
                p.multiProcessorCount, p.clockRate / 1000);
    uint32_t *out = nullptr;
    if (hipMalloc(&out, sizeof(uint32_t) * kBlocks * kThreads) != hipSuccess) return 1;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    all<0>(out, e0, e1);
    (void)hipFree(out);
    return 0;
}
