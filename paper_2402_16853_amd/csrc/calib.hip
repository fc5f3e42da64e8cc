// Calibration kernels for the roofline of the RQA tile kernel.  (1) The
// sustained issue rate of exactly the predicate's instruction stream (L-infinity, m = 3:
// three v_sub_f32 with a scalar operand, v_max3_f32 with |x| modifiers, one
// v_sub_f32 from the threshold in a VGPR and one v_alignbit_b32 per column; column coordinates from
// s_load_dwordx16), with nothing else in the loop.  (2) The LDS read
// bandwidth with conflict-free 16-byte reads.  Built into libcalib.so and used
// only by bench.py --probe-valu / --probe-lds.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef const __attribute__((address_space(4))) float *ConstF;

constexpr int kSeries = 4096;   // floats of the synthetic series
constexpr int kTau = 10;

// 64-column predicate tile of one lane's row, as in the tile kernel.
__device__ __forceinline__ uint32_t tile16(ConstF cb, float x0, float x1, float x2, float thr,
                                           uint32_t acc) {
#pragma unroll
    for (int b = 15; b >= 0; --b) {
        const float a = fmaxf(fmaxf(fabsf(cb[b] - x0), fabsf(cb[b + kTau] - x1)),
                              fabsf(cb[b + 2 * kTau] - x2));
        acc = __builtin_amdgcn_alignbit(acc, __float_as_uint(thr - a), 31);
    }
    return acc;
}

__global__ void __launch_bounds__(512) k_predicate_only(const float *__restrict__ s, int iters,
                                                        float thr, uint32_t *out) {
    const int lane = threadIdx.x;
    const float x0 = s[lane & 1023], x1 = s[(lane + kTau) & 1023], x2 = s[(lane + 2 * kTau) & 1023];
    const ConstF cs = (ConstF)(s);
    uint32_t acc = 0, sink = 0;
    asm volatile("" : "+v"(thr));   // threshold in a VGPR, as in the tile kernel
    int base = __builtin_amdgcn_readfirstlane(blockIdx.x * 16) & 2047;
    for (int it = 0; it < iters; ++it) {
        acc = tile16(cs + base, x0, x1, x2, thr, acc);
        sink ^= acc;
        base = (base + 16) & 2047;
    }
    if (sink == 0x9E3779B9u) out[lane] = sink;   // keeps the work observable
}

// LDS read rate: each lane reads 16 bytes per step (ds_read_b128) at addresses
// that cover all banks without conflicts; 64 KB of LDS per workgroup.
__global__ void __launch_bounds__(1024) k_lds_read(int iters, uint32_t *out) {
    __shared__ uint4 buf[4096];
    for (int t = threadIdx.x; t < 4096; t += blockDim.x)
        buf[t] = make_uint4(t, t * 3u, t * 5u, t * 7u);
    __syncthreads();
    uint32_t acc = 0;
    int idx = threadIdx.x & 4095;
    for (int it = 0; it < iters; ++it) {
        const uint4 v = buf[idx];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
        idx = (idx + 64) & 4095;
    }
    if (acc == 0x9E3779B9u) out[threadIdx.x] = acc;   // keeps the work observable
}

}  // namespace

extern "C" {

// LDS read bandwidth probe: `blocks` x `threads` lanes each read 16 bytes per
// step for `iters` steps; elapsed milliseconds returned in *ms.
int calib_lds(int blocks, int threads, int iters, double *ms) {
    uint32_t *out = nullptr;
    if (hipMalloc(&out, 1024 * sizeof(uint32_t)) != hipSuccess) return -1;
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(threads), 0, 0, 16, out);
    hipEventRecord(a, 0);
    hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(threads), 0, 0, iters, out);
    hipEventRecord(b, 0);
    hipEventSynchronize(b);
    float t = 0.f;
    hipEventElapsedTime(&t, a, b);
    *ms = t;
    hipEventDestroy(a);
    hipEventDestroy(b);
    hipFree(out);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Launch `blocks` workgroups of `threads` (multiple of 64) for `iters` chunks of
// 16 columns each and return the elapsed milliseconds (hipEvents).  Each chunk
// is 16 columns x 6 VALU instructions per wave.
int calib_predicate(int blocks, int threads, int iters, double *ms) {
    float *s = nullptr;
    uint32_t *out = nullptr;
    if (hipMalloc(&s, kSeries * sizeof(float)) != hipSuccess) return -1;
    if (hipMalloc(&out, 512 * sizeof(uint32_t)) != hipSuccess) return -1;
    float h[kSeries];
    for (int k = 0; k < kSeries; ++k) h[k] = (float)((k * 2654435761u) % 1000u) * 1e-3f;
    hipMemcpy(s, h, sizeof h, hipMemcpyHostToDevice);
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    hipLaunchKernelGGL(k_predicate_only, dim3(blocks), dim3(threads), 0, 0, s, 16, 0.3f, out);
    hipEventRecord(a, 0);
    hipLaunchKernelGGL(k_predicate_only, dim3(blocks), dim3(threads), 0, 0, s, iters, 0.3f, out);
    hipEventRecord(b, 0);
    hipEventSynchronize(b);
    float t = 0.f;
    hipEventElapsedTime(&t, a, b);
    *ms = t;
    hipEventDestroy(a);
    hipEventDestroy(b);
    hipFree(s);
    hipFree(out);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"
