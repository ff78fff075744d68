// Sketch of an arrival-order event stream (Section 2: the sketch is updated online as each
// photon arrives).  Events (pixel, stamp) come in any order; the sketch of a pixel is the sum
// over its events, so the stream is first grouped by pixel on the device -- a counting sort:
// photons per pixel (integer atomics), their exclusive prefix sums (the CSR offsets), and a
// scatter of every stamp into its pixel's range -- and then sketched by the binned pass.  The
// binned pass sums exact integer histograms, so the order in which the scatter places a pixel's
// stamps does not change the result (a pixel whose bin passes 255 is recomputed in chunks of
// the stored order; its rounding then follows that order, within the same error bound).
#include <algorithm>

#include "common.hpp"

namespace srt3d {

namespace {

constexpr int kEvThreads = 256;
constexpr int kScanPer = 4;                              // counts per thread in the scan
constexpr int kScanBlock = kEvThreads * kScanPer;        // counts per scan workgroup

__global__ __launch_bounds__(kEvThreads) void zero_counts_kernel(int32_t* __restrict__ counts, int P) {
    for (int64_t i = (int64_t)blockIdx.x * kEvThreads + threadIdx.x; i < P; i += (int64_t)gridDim.x * kEvThreads)
        counts[i] = 0;
}

// Photons per pixel; events whose pixel lies outside [0, P) are counted in err[1].
__global__ __launch_bounds__(kEvThreads) void count_events_kernel(const int32_t* __restrict__ pix, int64_t N, int P,
                                                                  int32_t* __restrict__ counts,
                                                                  int32_t* __restrict__ err) {
    int bad = 0;
    for (int64_t e = (int64_t)blockIdx.x * kEvThreads + threadIdx.x; e < N; e += (int64_t)gridDim.x * kEvThreads) {
        const int32_t p = pix[e];
        if ((uint32_t)p < (uint32_t)P) atomicAdd(&counts[p], 1);
        else ++bad;
    }
    if (err) {
        for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && bad) atomicAdd(&err[1], bad);
    }
}

// Exclusive scan of the workgroup's thread sums in LDS (Hillis-Steele over kEvThreads entries).
__device__ int64_t block_exclusive(int64_t v, int64_t* s) {
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kEvThreads; o <<= 1) {
        const int64_t add = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    const int64_t incl = s[threadIdx.x];
    __syncthreads();
    return incl - v;
}

// Sum of each block of kScanBlock counts.
__global__ __launch_bounds__(kEvThreads) void block_sums_kernel(const int32_t* __restrict__ counts, int P,
                                                                int64_t* __restrict__ bsum) {
    __shared__ int64_t s[kEvThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    int64_t v = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < P) v += counts[base + i];
    const int64_t ex = block_exclusive(v, s);
    if (threadIdx.x == kEvThreads - 1) bsum[blockIdx.x] = ex + v;
}

// Exclusive prefix of the block sums, in place (one workgroup, chunk by chunk).
__global__ __launch_bounds__(kEvThreads) void block_prefix_kernel(int64_t* __restrict__ bsum, int nb) {
    __shared__ int64_t s[kEvThreads];
    int64_t carry = 0;
    for (int c0 = 0; c0 < nb; c0 += kEvThreads) {
        const int i = c0 + threadIdx.x;
        const int64_t v = i < nb ? bsum[i] : 0;
        const int64_t ex = block_exclusive(v, s);
        if (i < nb) bsum[i] = carry + ex;
        if (threadIdx.x == kEvThreads - 1) s[0] = ex + v;      // the chunk's total
        __syncthreads();
        carry += s[0];
        __syncthreads();
    }
}

// offsets[p + 1] = sum of counts[0..p], offsets[0] = 0.
__global__ __launch_bounds__(kEvThreads) void write_offsets_kernel(const int32_t* __restrict__ counts, int P,
                                                                   const int64_t* __restrict__ bprefix,
                                                                   int64_t* __restrict__ offsets) {
    __shared__ int64_t s[kEvThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
    int32_t c[kScanPer];
    int64_t v = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        c[i] = base + i < P ? counts[base + i] : 0;
        v += c[i];
    }
    int64_t run = bprefix[blockIdx.x] + block_exclusive(v, s);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        run += c[i];
        if (base + i < P) offsets[base + i + 1] = run;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) offsets[0] = 0;
}

// Each stamp into its pixel's range: counts[p] counts down from the pixel's total, so the
// stamps fill offsets[p] .. offsets[p + 1] - 1 (in an order set by the atomics).
__global__ __launch_bounds__(kEvThreads) void scatter_events_kernel(const int32_t* __restrict__ pix,
                                                                    const int32_t* __restrict__ stamps, int64_t N,
                                                                    int P, const int64_t* __restrict__ offsets,
                                                                    int32_t* __restrict__ counts,
                                                                    int32_t* __restrict__ sorted) {
    for (int64_t e = (int64_t)blockIdx.x * kEvThreads + threadIdx.x; e < N; e += (int64_t)gridDim.x * kEvThreads) {
        const int32_t p = pix[e];
        if ((uint32_t)p >= (uint32_t)P) continue;
        const int32_t left = atomicSub(&counts[p], 1);
        const int64_t pos = offsets[p] + left - 1;
        if (left >= 1 && pos < offsets[p + 1]) sorted[pos] = stamps[e];   // guards a stream changed between passes
    }
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t events_ws_bytes(int64_t N, int P) {
    const int64_t nb = ((int64_t)P + kScanBlock - 1) / kScanBlock;
    return align256((size_t)P * 4) + align256((size_t)nb * 8) + align256((size_t)(P + 1) * 8) +
           align256((size_t)(N > 0 ? N : 1) * 4);
}

hipError_t launch_sketch_events(const int32_t* pix, const int32_t* stamps, int64_t N, int P, int T, int m,
                                const float2* table, float* z, int32_t* n, double* acc, int64_t* nacc, int32_t* err,
                                void* ws, hipStream_t s) {
    const int64_t nb = ((int64_t)P + kScanBlock - 1) / kScanBlock;
    char* w = reinterpret_cast<char*>(ws);
    int32_t* counts = reinterpret_cast<int32_t*>(w);
    w += align256((size_t)P * 4);
    int64_t* bsum = reinterpret_cast<int64_t*>(w);
    w += align256((size_t)nb * 8);
    int64_t* offsets = reinterpret_cast<int64_t*>(w);
    w += align256((size_t)(P + 1) * 8);
    int32_t* sorted = reinterpret_cast<int32_t*>(w);

    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    const int64_t stream_blocks = std::max<int64_t>(1, std::min<int64_t>((N + kEvThreads - 1) / kEvThreads,
                                                                         (int64_t)cus * 16));
    const int64_t pix_blocks = std::max<int64_t>(1, std::min<int64_t>((P + kEvThreads - 1) / kEvThreads,
                                                                      (int64_t)cus * 16));
    hipLaunchKernelGGL(zero_counts_kernel, dim3((unsigned)pix_blocks), dim3(kEvThreads), 0, s, counts, P);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (N > 0) {
        hipLaunchKernelGGL(count_events_kernel, dim3((unsigned)stream_blocks), dim3(kEvThreads), 0, s, pix, N, P, counts,
                           err);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(block_sums_kernel, dim3((unsigned)nb), dim3(kEvThreads), 0, s, counts, P, bsum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(block_prefix_kernel, dim3(1), dim3(kEvThreads), 0, s, bsum, (int)nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(write_offsets_kernel, dim3((unsigned)nb), dim3(kEvThreads), 0, s, counts, P, bsum, offsets);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (N > 0) {
        hipLaunchKernelGGL(scatter_events_kernel, dim3((unsigned)stream_blocks), dim3(kEvThreads), 0, s, pix, stamps, N,
                           P, offsets, counts, sorted);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // the grouped stream is an ordinary CSR frame of at most N stamps
    if (m <= 32) return launch_sketch_binned(sorted, N, offsets, P, T, m, table, z, n, acc, nacc, err, s);
    return launch_sketch_photons(sorted, N, offsets, P, T, m, table, z, n, acc, nacc, err, s);
}

}  // namespace srt3d
