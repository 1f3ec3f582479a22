// Microbenchmarks that measure the hardware rates the PIC kernels are bound
// by on gfx950: LDS FP32 / FP64 atomic adds and LDS reads under several
// lane-to-address patterns, global FP64 atomic adds, HBM copy bandwidth,
// and the field-stage copy (row segments into LDS) by lines per row.  Each entry point times its own kernel with HIP events and
// returns milliseconds (negative on a HIP error).  Used by
// paper_2303_12873_amd/microbench.py; not part of the PIC step.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace {

constexpr int MB_BLOCK = 512;
constexpr int MB_LDS_WORDS = 8192;   // 32 KB of 4-byte words

// Lane -> LDS slot.  pattern 0: distinct consecutive slots; 1: groups of 4
// consecutive lanes share a slot; 2: every lane of the wave the same slot;
// 3: distinct slots two words apart; 4: distinct slots 15 words apart;
// 5 / 6: the lanes of a wave on an 8 x 8 block of cells of a tile whose rows
// are 15 / 24 slots long (the current tile's row without / with padding);
// 7 / 8: on a 16 x 4 block, rows 23 / 24 long; 9 / 10: the same with lane
// bits 4 and 5 swapped (a half-wave on rows r and r + 2).
__device__ inline int slot(int lane, int wave, int pattern) {
    const int sw = lane ^ ((((lane >> 4) ^ (lane >> 5)) & 1) * 48);
    switch (pattern) {
        case 0: return wave * 64 + lane;
        case 1: return wave * 16 + lane / 4;
        case 2: return wave;
        case 3: return wave * 128 + 2 * lane;
        case 4: return (wave * 64 + lane) * 15 % 4096;
        case 5: return (lane & 7) + 15 * (lane >> 3) + 3 * wave;
        case 6: return (lane & 7) + 24 * (lane >> 3) + 3 * wave;
        case 7: return (lane & 15) + 23 * (lane >> 4) + 3 * wave;
        case 8: return (lane & 15) + 24 * (lane >> 4) + 3 * wave;
        case 9: return (sw & 15) + 23 * (sw >> 4) + 3 * wave;
        default: return (sw & 15) + 24 * (sw >> 4) + 3 * wave;
    }
}

template <typename T>
__global__ void __launch_bounds__(MB_BLOCK) k_lds_atomic(int iters, int pattern, T *out) {
    __shared__ T lds[MB_LDS_WORDS * 4 / sizeof(T)];
    for (int i = threadIdx.x; i < (int)(MB_LDS_WORDS * 4 / sizeof(T)); i += blockDim.x) lds[i] = T(0);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int s = slot(lane, wave, pattern) % (MB_LDS_WORDS * 4 / (int)sizeof(T) / 2);
    const T v = T(1);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if constexpr (std::is_integral<T>::value) atomicAdd(&lds[s + u * 8], v);
            else unsafeAtomicAdd(&lds[s + u * 8], v);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = lds[s];
}

template <typename T>
__global__ void __launch_bounds__(MB_BLOCK) k_lds_read(int iters, int pattern, T *out) {
    __shared__ T lds[MB_LDS_WORDS * 4 / sizeof(T)];
    for (int i = threadIdx.x; i < (int)(MB_LDS_WORDS * 4 / sizeof(T)); i += blockDim.x) lds[i] = T(i & 7);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int s = slot(lane, wave, pattern) % (MB_LDS_WORDS * 4 / (int)sizeof(T) / 2);
    T acc = T(0);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += lds[s + u * 8];
        s ^= (it & 1);   // keep the loads inside the loop
    }
    if (acc == T(-1)) out[blockIdx.x] = acc;
}

__global__ void k_global_atomic(double *buf, long long nslots, int iters, int collide) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long s = collide ? (t / 64) % nslots : t % nslots;
    for (int it = 0; it < iters; ++it) unsafeAtomicAdd(&buf[s], 1.0);
}

__global__ void k_copy16(const int4 *__restrict__ src, int4 *__restrict__ dst, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[i];
}

// The field-stage copy pattern: each workgroup (one per CU, 1024 threads)
// copies `rows` row segments of `len` floats, row r at element
// r * row_stride + start of its own source region, into consecutive LDS
// words with global -> LDS loads, `reps` times (a wait and a barrier after
// each), and records the device wall clock around the loop.
__global__ void __launch_bounds__(1024) k_stage_rows(const float *src, long long wg_stride, int rows,
                                                     int len, int start, int row_stride, int reps,
                                                     unsigned long long *ticks) {
    extern __shared__ __attribute__((aligned(16))) float stage[];
    const float *base = src + blockIdx.x * wg_stride;
    const int n = rows * len;
    const int lane = threadIdx.x & 63;
    const unsigned long long t0 = wall_clock64();
    for (int r = 0; r < reps; ++r) {
        for (int id = threadIdx.x; id < n; id += blockDim.x) {
            const int row = id / len, i = id - row * len;
            __builtin_amdgcn_global_load_lds(
                (const unsigned *)(base + (long long)row * row_stride + start + i),
                (unsigned *)stage + (id - lane), 4, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    if (threadIdx.x == 0) ticks[blockIdx.x] = wall_clock64() - t0;
}

// The same copy with `width` bytes per lane (4, 12 or 16: one, three or
// four dwords of a row per lane; len a multiple of width / 4); block 0
// writes its LDS words back to `check` after the last copy so that the
// lane -> LDS layout can be compared with the source on the host.
template <int WIDTH>
__global__ void __launch_bounds__(1024) k_stage_rows_w(const float *src, long long wg_stride, int rows,
                                                       int len, int start, int row_stride, int reps,
                                                       int lds_off, unsigned long long *ticks,
                                                       float *check) {
    extern __shared__ __attribute__((aligned(16))) float lds_all[];
    float *stage = lds_all + lds_off;       // LDS words from lds_off on
    constexpr int V = WIDTH / 4;             // floats per lane
    const float *base = src + blockIdx.x * wg_stride;
    const int per_row = len / V;            // lanes per row
    const int n = rows * per_row;
    const int lane = threadIdx.x & 63;
    const unsigned long long t0 = wall_clock64();
    for (int r = 0; r < reps; ++r) {
        for (int id = threadIdx.x; id < n; id += blockDim.x) {
            const int row = id / per_row, i = (id - row * per_row) * V;
            const unsigned *g = (const unsigned *)(base + (long long)row * row_stride + start + i);
            unsigned *l = (unsigned *)stage + (id - lane) * V;
            if constexpr (WIDTH == 4) __builtin_amdgcn_global_load_lds(g, l, 4, 0, 0);
            else if constexpr (WIDTH == 12) __builtin_amdgcn_global_load_lds(g, l, 12, 0, 0);
            else __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    if (threadIdx.x == 0) ticks[blockIdx.x] = wall_clock64() - t0;
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < rows * len; k += blockDim.x) check[k] = stage[k];
}

template <typename F>
float time_ms(F launch, int reps) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0f;
    launch();
    (void)hipDeviceSynchronize();
    (void)hipEventRecord(a, 0);
    for (int r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(b, 0);
    (void)hipEventSynchronize(b);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (hipGetLastError() != hipSuccess) return -1.0f;
    return ms / reps;
}

}  // namespace

extern "C" {

// LDS atomics (kind 0) or reads (kind 1) of FP32 (bytes 4) or FP64
// (bytes 8), or integer atomic adds (kind 2) of 32-bit (bytes 4) or 64-bit
// (bytes 8) integers: `blocks` workgroups of 512 threads, each lane issuing
// 8 * iters operations.  Returns ms per launch.
float pic_mb_lds(int kind, int bytes, int pattern, int blocks, int iters) {
    void *out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 8) != hipSuccess) return -1.0f;
    float ms;
    if (kind == 2 && bytes == 4)
        ms = time_ms([&] { hipLaunchKernelGGL(k_lds_atomic<unsigned int>, dim3(blocks), dim3(MB_BLOCK), 0, 0, iters, pattern, (unsigned int *)out); }, 3);
    else if (kind == 2)
        ms = time_ms([&] { hipLaunchKernelGGL(k_lds_atomic<unsigned long long>, dim3(blocks), dim3(MB_BLOCK), 0, 0, iters, pattern, (unsigned long long *)out); }, 3);
    else if (kind == 0 && bytes == 4)
        ms = time_ms([&] { hipLaunchKernelGGL(k_lds_atomic<float>, dim3(blocks), dim3(MB_BLOCK), 0, 0, iters, pattern, (float *)out); }, 3);
    else if (kind == 0)
        ms = time_ms([&] { hipLaunchKernelGGL(k_lds_atomic<double>, dim3(blocks), dim3(MB_BLOCK), 0, 0, iters, pattern, (double *)out); }, 3);
    else if (bytes == 4)
        ms = time_ms([&] { hipLaunchKernelGGL(k_lds_read<float>, dim3(blocks), dim3(MB_BLOCK), 0, 0, iters, pattern, (float *)out); }, 3);
    else
        ms = time_ms([&] { hipLaunchKernelGGL(k_lds_read<double>, dim3(blocks), dim3(MB_BLOCK), 0, 0, iters, pattern, (double *)out); }, 3);
    (void)hipFree(out);
    return ms;
}

// Global FP64 atomic adds: `threads` threads x `iters` adds onto `nslots`
// distinct doubles (collide = 0) or one slot per wave (collide = 1).
float pic_mb_global_atomic(long long threads, long long nslots, int iters, int collide) {
    double *buf = nullptr;
    if (hipMalloc(&buf, (size_t)nslots * 8) != hipSuccess) return -1.0f;
    (void)hipMemset(buf, 0, (size_t)nslots * 8);
    int blocks = (int)((threads + 255) / 256);
    float ms = time_ms([&] { hipLaunchKernelGGL(k_global_atomic, dim3(blocks), dim3(256), 0, 0, buf, nslots, iters, collide); }, 3);
    (void)hipFree(buf);
    return ms;
}

// Device-to-device copy of `bytes` (multiple of 16) by a grid-stride kernel.
float pic_mb_copy(long long bytes, int blocks) {
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, (size_t)bytes) != hipSuccess) return -1.0f;
    if (hipMalloc(&b, (size_t)bytes) != hipSuccess) { (void)hipFree(a); return -1.0f; }
    (void)hipMemset(a, 1, (size_t)bytes);
    long long n = bytes / 16;
    float ms = time_ms([&] { hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(256), 0, 0, (const int4 *)a, (int4 *)b, n); }, 5);
    (void)hipFree(a);
    (void)hipFree(b);
    return ms;
}

// The field-stage pattern (k_stage_rows) on `blocks` workgroups, one per CU
// (100 KB of LDS each): returns the mean device wall-clock ticks (100 MHz)
// of `reps` stages per workgroup, negative on an error or on arguments that
// would reach past the LDS words written (rows * len <= 16384) or the
// source buffer.
double pic_mb_stage_rows(int blocks, int rows, int len, int start, int row_stride, int reps) {
    if (blocks < 1 || rows < 1 || len < 1 || start < 0 || row_stride < start + len || reps < 1 ||
        (long long)rows * len > 16384)
        return -1.0;
    const long long wg_stride = (long long)rows * row_stride + 64;
    float *src = nullptr;
    unsigned long long *ticks = nullptr;
    if (hipMalloc(&src, (size_t)(wg_stride * blocks) * sizeof(float)) != hipSuccess) return -1.0;
    if (hipMalloc(&ticks, (size_t)blocks * 8) != hipSuccess) { (void)hipFree(src); return -1.0; }
    (void)hipMemset(src, 0, (size_t)(wg_stride * blocks) * sizeof(float));
    const int lds = 100 * 1024;
    double mean = -1.0;
    if (hipFuncSetAttribute((const void *)&k_stage_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds) == hipSuccess) {
        hipLaunchKernelGGL(k_stage_rows, dim3(blocks), dim3(1024), lds, 0, (const float *)src,
                           wg_stride, rows, len, start, row_stride, reps, ticks);
        if (hipDeviceSynchronize() == hipSuccess && hipGetLastError() == hipSuccess) {
            unsigned long long *h = new unsigned long long[blocks];
            if (hipMemcpy(h, ticks, (size_t)blocks * 8, hipMemcpyDeviceToHost) == hipSuccess) {
                double sum = 0.0;
                for (int b = 0; b < blocks; ++b) sum += (double)h[b];
                mean = sum / blocks / reps;
            }
            delete[] h;
        }
    }
    (void)hipFree(src);
    (void)hipFree(ticks);
    return mean;
}

// k_stage_rows_w: `width` bytes per lane (4, 12, 16), the copies landing
// at LDS word `lds_off` on (a multiple of 4; lds_off + rows * len <= 24576,
// inside the 100 KB allocation whatever part of the address the loads
// honour); source element e holds the value e, and `check` (rows * len
// floats, host memory) receives workgroup 0's LDS words from lds_off.
// Returns mean ticks per stage as above.
double pic_mb_stage_rows_w(int width, int blocks, int rows, int len, int start, int row_stride,
                           int reps, int lds_off, float *check) {
    if ((width != 4 && width != 12 && width != 16) || blocks < 1 || rows < 1 || len < 1 ||
        len % (width / 4) != 0 || start < 0 || row_stride < start + len || reps < 1 ||
        lds_off < 0 || lds_off % 4 != 0 || (long long)rows * len > 16384 ||
        lds_off + (long long)rows * len > 24576)
        return -1.0;
    const long long wg_stride = (long long)rows * row_stride + 64;
    const long long nsrc = wg_stride * blocks;
    float *src = nullptr, *dcheck = nullptr;
    unsigned long long *ticks = nullptr;
    if (hipMalloc(&src, (size_t)nsrc * sizeof(float)) != hipSuccess) return -1.0;
    if (hipMalloc(&ticks, (size_t)blocks * 8) != hipSuccess) { (void)hipFree(src); return -1.0; }
    if (hipMalloc(&dcheck, (size_t)rows * len * sizeof(float)) != hipSuccess) {
        (void)hipFree(src); (void)hipFree(ticks); return -1.0;
    }
    {
        float *h = new float[nsrc];
        for (long long e = 0; e < nsrc; ++e) h[e] = (float)(e % 16777216);
        (void)hipMemcpy(src, h, (size_t)nsrc * sizeof(float), hipMemcpyHostToDevice);
        delete[] h;
    }
    const int lds = 100 * 1024;
    double mean = -1.0;
    hipError_t e = hipSuccess;
    if (width == 4)
        e = hipFuncSetAttribute((const void *)&k_stage_rows_w<4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    else if (width == 12)
        e = hipFuncSetAttribute((const void *)&k_stage_rows_w<12>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    else
        e = hipFuncSetAttribute((const void *)&k_stage_rows_w<16>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess) {
        if (width == 4)
            hipLaunchKernelGGL(k_stage_rows_w<4>, dim3(blocks), dim3(1024), lds, 0, (const float *)src,
                               wg_stride, rows, len, start, row_stride, reps, lds_off, ticks, dcheck);
        else if (width == 12)
            hipLaunchKernelGGL(k_stage_rows_w<12>, dim3(blocks), dim3(1024), lds, 0, (const float *)src,
                               wg_stride, rows, len, start, row_stride, reps, lds_off, ticks, dcheck);
        else
            hipLaunchKernelGGL(k_stage_rows_w<16>, dim3(blocks), dim3(1024), lds, 0, (const float *)src,
                               wg_stride, rows, len, start, row_stride, reps, lds_off, ticks, dcheck);
        if (hipDeviceSynchronize() == hipSuccess && hipGetLastError() == hipSuccess) {
            unsigned long long *h = new unsigned long long[blocks];
            if (hipMemcpy(h, ticks, (size_t)blocks * 8, hipMemcpyDeviceToHost) == hipSuccess &&
                hipMemcpy(check, dcheck, (size_t)rows * len * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess) {
                double sum = 0.0;
                for (int b = 0; b < blocks; ++b) sum += (double)h[b];
                mean = sum / blocks / reps;
            }
            delete[] h;
        }
    }
    (void)hipFree(src);
    (void)hipFree(ticks);
    (void)hipFree(dcheck);
    return mean;
}

}  // extern "C"
