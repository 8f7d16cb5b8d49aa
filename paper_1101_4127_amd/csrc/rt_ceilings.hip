// rt_ceilings.hip -- microbenchmarks of the ceilings the packet march runs
// against (include/rt_ceilings.h): HBM copy and read bandwidth, float64
// atomic adds into device memory and into LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rt_ceilings.h"

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    // integer hash (xor-shift-multiply rounds) spreading consecutive keys
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(kBlock) k_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src, size_t n) {
    const size_t stride = (size_t)gridDim.x * kBlock;
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

__global__ void __launch_bounds__(kBlock) k_read(const float4 *__restrict__ src, size_t n, float *sink) {
    const size_t stride = (size_t)gridDim.x * kBlock;
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    float acc = 0.0f;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        acc += (a.x + b.y) + (c.z + d.w);
    }
    for (; i < n; i += stride) acc += src[i].x;
    __shared__ float red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) sink[blockIdx.x & 65535u] = red[0];
}

__global__ void __launch_bounds__(kBlock) k_global_atomic(double *buf, uint32_t mask, uint32_t per) {
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t idx = mix32(t * per + k) & mask;
        unsafeAtomicAdd(buf + idx, 1.0);
    }
}

__global__ void __launch_bounds__(kBlock) k_lds_atomic(int acc, int soa, uint32_t per, double *sink) {
    __shared__ double s[512 * 4];
    for (int i = threadIdx.x; i < 512 * 4; i += kBlock) s[i] = 0.0;
    __syncthreads();
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t cell = mix32(t * per + k) & 511u;
        for (int a = 0; a < acc; ++a) {
            const uint32_t idx = soa ? (uint32_t)a * 512u + cell : cell * (uint32_t)acc + (uint32_t)a;
            atomicAdd(s + idx, 1.0);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int i = 0; i < 512 * acc; ++i) v += s[i];
        sink[blockIdx.x & 65535u] = v;
    }
}

int cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return n;
}

// Time `launch` (enqueued reps times after one untimed run) on the stream.
template <typename F>
int32_t timed(hipStream_t st, int reps, F launch, double *ms) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -3;
    launch();
    bool ok = hipEventRecord(a, st) == hipSuccess;
    for (int r = 0; r < reps && ok; ++r) {
        launch();
        ok = hipGetLastError() == hipSuccess;
    }
    float t = 0.0f;
    ok = ok && hipEventRecord(b, st) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
         hipEventElapsedTime(&t, a, b) == hipSuccess;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (!ok) return -3;
    *ms = t;
    return 0;
}

}  // namespace

extern "C" {

int32_t rtc_hbm_copy(void *d_dst, const void *d_src, size_t bytes, int32_t reps, void *hip_stream, double *gbs) {
    if (!d_dst || !d_src || !gbs || bytes == 0 || bytes % 16 || reps < 1) return -1;
    if ((reinterpret_cast<uintptr_t>(d_dst) | reinterpret_cast<uintptr_t>(d_src)) % 16) return -1;
    const int n = cus();
    if (n < 1) return -3;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const size_t nv = bytes / 16;
    double ms = 0.0;
    const int32_t r = timed(st, reps, [&] {
        hipLaunchKernelGGL(k_copy, dim3(n * 8), dim3(kBlock), 0, st, reinterpret_cast<uint4 *>(d_dst),
                           reinterpret_cast<const uint4 *>(d_src), nv);
    }, &ms);
    if (r) return r;
    *gbs = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return 0;
}

int32_t rtc_hbm_read(const void *d_src, size_t bytes, int32_t reps, float *d_sink, void *hip_stream, double *gbs) {
    if (!d_src || !d_sink || !gbs || bytes == 0 || bytes % 16 || reps < 1) return -1;
    if (reinterpret_cast<uintptr_t>(d_src) % 16) return -1;
    const int n = cus();
    if (n < 1) return -3;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const size_t nv = bytes / 16;
    double ms = 0.0;
    const int32_t r = timed(st, reps, [&] {
        hipLaunchKernelGGL(k_read, dim3(n * 8), dim3(kBlock), 0, st, reinterpret_cast<const float4 *>(d_src), nv,
                           d_sink);
    }, &ms);
    if (r) return r;
    *gbs = (double)bytes * reps / (ms * 1e-3) / 1e9;
    return 0;
}

int32_t rtc_global_atomic_f64(double *d_buf, size_t n, int64_t updates, void *hip_stream, double *rate) {
    if (!d_buf || !rate || n == 0 || (n & (n - 1)) || n > ((size_t)1 << 32) || updates < 1) return -1;
    const int c = cus();
    if (c < 1) return -3;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const uint32_t blocks = (uint32_t)c * 8u;
    const int64_t threads = (int64_t)blocks * kBlock;
    const int64_t per = (updates + threads - 1) / threads;
    if (per > 0x7fffffff) return -1;
    double ms = 0.0;
    const int32_t r = timed(st, 1, [&] {
        hipLaunchKernelGGL(k_global_atomic, dim3(blocks), dim3(kBlock), 0, st, d_buf, (uint32_t)(n - 1),
                           (uint32_t)per);
    }, &ms);
    if (r) return r;
    *rate = (double)(per * threads) / (ms * 1e-3);
    return 0;
}

int32_t rtc_lds_atomic_f64(int32_t acc, int32_t soa, int64_t updates, double *d_sink, void *hip_stream,
                           double *rate) {
    if (!d_sink || !rate || acc < 1 || acc > 4 || (soa != 0 && soa != 1) || updates < 1) return -1;
    const int c = cus();
    if (c < 1) return -3;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const uint32_t blocks = (uint32_t)c * 4u;
    const int64_t visits = (updates + acc - 1) / acc;
    const int64_t threads = (int64_t)blocks * kBlock;
    const int64_t per = (visits + threads - 1) / threads;
    if (per > 0x7fffffff) return -1;
    double ms = 0.0;
    const int32_t r = timed(st, 1, [&] {
        hipLaunchKernelGGL(k_lds_atomic, dim3(blocks), dim3(kBlock), 0, st, (int)acc, (int)soa, (uint32_t)per,
                           d_sink);
    }, &ms);
    if (r) return r;
    *rate = (double)(per * threads * acc) / (ms * 1e-3);
    return 0;
}

}  // extern "C"
